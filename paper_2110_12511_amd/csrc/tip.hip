// Tip decomposition by two-phase peeling (Section 3.2).
//
// X is the peeled side, Y the other side (X = U, or X = V on the transposed
// view).  Butterflies hold exactly two X-vertices, so peeling an active set
// changes each surviving x' by the sum over active x of C(c(x,x'), 2), with
// c the common-neighbour count; these updates from different active vertices
// are disjoint butterflies and aggregate with plain atomics (Section 3.2).
//
// Coarse-grained phase (Algorithm 4 structure, tip form): per partition i,
//   * work w_x = sum over y in N_x of the live degree of y (the wedge count
//     of x, also the quantity of the batch rule in Section 5.1);
//   * bound theta(i+1) = 1 + the smallest support whose cumulative alive work
//     reaches the adaptive target (find_range);
//   * support snapshot (the initialisation vector) and the first active set;
//   * rounds: peel the active set by wedge traversal (or recount the remaining
//     graph when the active set's wedges exceed the counting bound,
//     Section 5.1); vertices whose support crosses below the bound form the
//     next active set; peeled vertices are dropped from the Y lists
//     (Section 5.2).
// Fine-grained phase: each partition is peeled alone on the subgraph induced
// by its vertices and all of Y, starting from the snapshot, in one persistent
// kernel whose workgroups pop partitions from a queue sorted by decreasing
// estimated work (Section 3.1.4).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "dev_common.h"
#include "pbng_internal.h"

namespace pbng {

enum : unsigned char { ST_ALIVE = 0, ST_ACTIVE = 1, ST_PEELED = 2 };

constexpr i64 T_SMALL_W = 512, T_MEDIUM_W = 4096;

struct TipCtl {
    u64 bound;      // theta(i+1)
    u64 s;          // selected support
    u64 est_init;   // estimated work of the partition when its bound was chosen
    u64 est_final;  // work of all vertices that joined the partition
    double scale;   // scaling factor for the next target
    u32 nF;         // current active-set size
    u32 nF2;        // next active-set size
    u64 wF;         // wedges of the current active set (live lists)
    u64 wedges;     // wedges walked by peeling kernels
    u32 nbin[5];    // active-set bins: small, medium, hash ranges, key tiles, pair intersections
    u32 next[5];    // work counters
    u32 ndirty;     // Y lists to compact
    i32 pid;        // current partition
    u64 tnext;      // work counter of the key-tile items (vertex x tile)
    u64 alive;      // vertices neither active nor peeled, before the round
    u64 wbound;     // recount bound on an active set's wedges (Section 5.1)
    u64 rounds;     // rounds with a nonempty active set (captured rounds)
    u32 recount;    // a captured round handed its active set to a recount
    u32 pad2;
};

// Captured coarse-grained rounds: a HIP graph of TIP_GRAPH_K rounds (even,
// so the current and next active-set buffers are back in place after a
// replay) is replayed until a partition's active set is empty.  Most
// partitions take two rounds: the one the frontier starts and a short one
// for the vertices it pushes below the bound.
constexpr int TIP_GRAPH_K = 2;

// Heavy active vertices accumulate c(x, x') in LDS over key tiles of
// 2^TILE_LOG consecutive X ids, two 16-bit counters per 32-bit word, or of
// 2^(TILE_LOG - 1) ids with 32-bit counters when a degree reaches 2^16.
constexpr int TILE_LOG = 16;
// active vertices with more wedges than this take the key-tile path
constexpr i64 HUGE_W = i64(1) << 16;
// LDS hash slots of the (vertex, key range) path, and its workgroups per CU
constexpr int H_LOGCAP = 13;
constexpr int H_BLOCK = 512;
constexpr int H_WG_PER_CU = 2;
// sets of HBM counters for the key-range kernel's overflow pass
constexpr u32 H_OVF = 8;
// active vertices with 2..PAIR_DMAX neighbours whose pairwise list
// intersections cost less than 1 / PAIR_COST of their wedges take that path
constexpr i64 PAIR_DMAX = 8;
// an alive set of at most this many vertices, with at least this much work
// in all and per vertex on average, is peeled one support level per
// partition (see tip_decompose)
constexpr i64 LEVEL_MAX_ALIVE = 1024;
constexpr u64 LEVEL_MIN_WORK = u64(1) << 30;
constexpr u64 LEVEL_MIN_AVG = u64(1) << 21;
constexpr u64 PAIR_COST = 4;

__device__ __forceinline__ int bits_of(u32 v) { return v ? 32 - __clz(v) : 0; }

struct PeelArgs {
    const i64 *xrow;
    const i32 *xadj;
    const i64 *yrow;
    const i32 *yadj;
    const i32 *ylen;
    const i32 *items;
    const u32 *nitems;
    u32 *next;
    const unsigned char *st;
    u64 *sup;
    const u64 *wi;       // wedges of each active vertex over the live lists
    const u64 *bound;
    i32 *nf;
    u32 *nnf;
    u32 *dcnt;           // key-range overflow: H_OVF sets of HBM counters (nx each, zero between holders)
    i32 *dtouch;         // their touched keys (nx each)
    u32 *dlock;          // one lock word per set
    i32 hprobe;          // LDS probe limit of the key-range path
    const i32 *kspan;    // key-range bin: smallest and largest X id in the vertex's live lists
    i32 ntiles;
    i64 nx;
    u64 *tnext;          // key-tile item counter
    u64 *wedges;
    KCounters *kc;
};

struct ItemSmem {
    i32 *pre;
    i64 *moff;
    i32 *wave;
    u64 *red;
    i64 *bcast;
};

// Every wedge x -> y -> x' of an active x over the live Y lists is counted
// per x'; then every x' with c >= 2 loses C(c, 2) of its support; after the
// round the alive vertices whose support fell below the bound form the next
// active set.
// Support updates of a batch of NB (key, count) pairs.  Keys < 0 or counts
// < 2 are skipped.  Keys that are not alive (other vertices active this
// round, and peeled ones when list compaction is off) are updated too: the
// support of a vertex is never read after it leaves the alive set (every
// reader filters on ST_ALIVE, and the fine-grained phase starts from the
// snapshot taken when its partition began), so the update is harmless and
// saves a dependent state load per key.  The subtractions are
// fire-and-forget atomics (no returned value to wait for): the next active
// set is found after the round by k_sweep_frontier, as every alive vertex
// whose support fell below the bound, the same set the crossings would give.
template <int NB>
__device__ __forceinline__ void apply_updates(const PeelArgs &a, u64 B, const i32 (&key)[NB], const u32 (&cnt)[NB],
                                              Tally &t) {
    (void)B;
    bool ok[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) ok[q] = key[q] >= 0 && cnt[q] >= 2;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (!ok[q]) continue;
        const u64 dd = (u64)cnt[q] * (u64)(cnt[q] - 1) / 2;
        atomicAdd((unsigned long long *)&a.sup[key[q]], (unsigned long long)(0ull - dd));
        ++t.atomics;
    }
}

// Far ends of the wedges k0 .. k0 + UNR - 1 of a chunk of neighbour lists
// whose wedge counts have inclusive prefix pre[0..last] and whose runs start
// at yadj[moff[l]]; wedges at or past tot give x (skipped by the caller).
// One binary search finds the list of k0; the rest of the run walks forward,
// reading the next prefix only where a list ends.  All UNR addresses are
// formed first and every load is issued unconditionally (a wedge past tot
// reads yadj[0], which exists whenever tot > 0), so the loads are in flight
// together and the thread waits once.
template <int UNR>
__device__ __forceinline__ void run_ends(const i32 *yadj, const i32 *pre, const i64 *moff, int last, i32 k0, i32 tot,
                                         i32 x, i32 (&xq)[UNR]) {
    i64 idx[UNR];
#pragma unroll
    for (int q = 0; q < UNR; ++q) idx[q] = 0;
    if (k0 < tot) {
        int l = 0, h = last;
        while (l < h) {
            const int md = (l + h) >> 1;
            if (pre[md] > k0) h = md; else l = md + 1;
        }
        i32 end = pre[l];
        i64 base = moff[l] - (l ? pre[l - 1] : 0);
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const i32 k = k0 + q;
            if (k < tot) {
                while (k >= end) {
                    ++l;
                    base = moff[l] - end;
                    end = pre[l];
                }
                idx[q] = base + k;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < UNR; ++q) xq[q] = yadj[idx[q]];
#pragma unroll
    for (int q = 0; q < UNR; ++q)
        if (k0 + q >= tot) xq[q] = x;
}

// Probe of one step of a lower-bound search over a[lo, hi) whose keys lie
// in [vlo, vhi) and which holds k in that range: the interpolated position
// while interp is set (keys spread evenly over the id space land within a
// few slots), the midpoint otherwise.
__device__ __forceinline__ i64 lb_probe(i64 lo, i64 hi, i64 vlo, i64 vhi, i64 k, bool interp) {
    i64 p;
    if (interp && vhi > vlo)
        p = lo + (i64)((u64)(k - vlo) * (u64)(hi - lo) / (u64)(vhi - vlo));
    else
        p = (lo + hi) >> 1;
    return p < hi ? p : hi - 1;
}

// Steps of a search that interpolate; later steps halve, so a search takes
// at most LB_INTERP + log2(run) + 1 dependent loads for any key spread.
constexpr int LB_INTERP = 6;

// The run of a sorted, duplicate-free live list a[base, end) of X ids
// (below nx) with ids in [k0, k1): p0 = first slot with id >= k0, p1 =
// first slot with id >= k1 (k0 <= k1; k0 <= 0 gives base, k1 >= nx gives
// end).  The two searches advance in lockstep, so the loads of one step of
// both are in flight together; each keeps the key interval of its slot
// interval, [vlo, vhi), for the interpolation.
__device__ __forceinline__ void run_bounds(const i32 *a, i64 base, i64 end, i64 nx, i64 k0, i64 k1, i64 &p0, i64 &p1) {
    i64 lo0 = base, hi0 = k0 > 0 ? end : base, vl0 = 0, vh0 = nx;
    i64 lo1 = k1 < nx ? base : end, hi1 = end, vl1 = 0, vh1 = nx;
    for (int it = 0; lo0 < hi0 || lo1 < hi1; ++it) {
        const bool ip = it < LB_INTERP;
        const bool a0 = lo0 < hi0, a1 = lo1 < hi1;
        const i64 q0 = a0 ? lb_probe(lo0, hi0, vl0, vh0, k0, ip) : 0;
        const i64 q1 = a1 ? lb_probe(lo1, hi1, vl1, vh1, k1, ip) : 0;
        const i64 v0 = a0 ? a[q0] : 0, v1 = a1 ? a[q1] : 0;
        if (a0) {
            if (v0 < k0) {
                lo0 = q0 + 1;
                vl0 = v0 + 1;
            } else {
                hi0 = q0;
                vh0 = v0;
            }
        }
        if (a1) {
            if (v1 < k1) {
                lo1 = q1 + 1;
                vl1 = v1 + 1;
            } else {
                hi1 = q1;
                vh1 = v1;
            }
        }
    }
    p0 = lo0;
    p1 = lo1;
}

// next active set of a push round: alive vertices below the bound (none
// when the round had no active set)
__global__ void k_sweep_frontier(const unsigned char *st, const u64 *sup, const TipCtl *ctl, i64 nx, i32 *nf, u32 *nnf) {
    if (ctl->nF == 0) return;
    const u64 B = ctl->bound;
    const i64 stride = (i64)gridDim.x * blockDim.x;
    const i64 nn = (nx + WAVE - 1) / WAVE * WAVE;
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nn; x += stride) {
        const bool take = x < nx && st[x] == ST_ALIVE && sup[x] < B;
        const u32 p = wave_append(nnf, take);
        if (take) nf[p] = (i32)x;
    }
}

template <int BLOCK, class Acc>
__device__ __forceinline__ void peel_item(const PeelArgs &a, i32 x, Acc &A, const ItemSmem &sm, Tally &t) {
    const i64 jb = a.xrow[x], je = a.xrow[x + 1];
    if (threadIdx.x == 0) {
        t.segments += (u64)(je - jb);
        t.items += 1;
    }
    for (i64 cb = jb; cb < je; cb += BLOCK) {
        i64 j = cb + threadIdx.x;
        i32 pl = 0;
        i64 moff = 0;
        if (j < je) {
            i32 y = a.xadj[j];
            pl = a.ylen[y];
            moff = a.yrow[y];
        }
        i32 tot;
        i32 incl = block_incl_scan_i32<BLOCK>(pl, sm.wave, tot);
        sm.pre[threadIdx.x] = incl;
        sm.moff[threadIdx.x] = moff;
        __syncthreads();
        for (i32 k = threadIdx.x; k < tot; k += BLOCK) {
            int lo = 0, hi = BLOCK - 1;
            while (lo < hi) {
                int md = (lo + hi) >> 1;
                if (sm.pre[md] > k) hi = md; else lo = md + 1;
            }
            i32 before = lo ? sm.pre[lo - 1] : 0;
            i32 xp = a.yadj[sm.moff[lo] + (k - before)];
            if (xp == x) continue;
            ++t.wedges;
            A.add(xp);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) sm.bcast[0] = A.entries();
    __syncthreads();
    const i64 ne = sm.bcast[0];
    __syncthreads();
    const u64 B = *a.bound;
    constexpr int NB = 4;
    for (i64 i0 = threadIdx.x; i0 < ne; i0 += (i64)NB * BLOCK) {
        i32 key[NB];
        u32 c32[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const i64 i = i0 + (i64)q * BLOCK;
            key[q] = -1;
            c32[q] = 0;
            if (i < ne) A.entry(i, key[q], c32[q]);
        }
        apply_updates<NB>(a, B, key, c32, t);
    }
    __syncthreads();
}

template <int BLOCK, int LOGCAP>
__global__ __launch_bounds__(BLOCK) void k_tip_peel_hash(PeelArgs a, int bin) {
    constexpr int CAP = 1 << LOGCAP;
    __shared__ i32 s_keys[CAP];
    __shared__ u32 s_vals[CAP];
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_red[BLOCK / WAVE];
    __shared__ i64 s_bcast[1];
    __shared__ i32 s_item;
    ItemSmem sm{s_pre, s_moff, s_wave, s_red, s_bcast};
    LdsAcc A;
    A.keys = s_keys;
    A.vals = s_vals;
    A.bids = nullptr;
    const u32 n = a.nitems[bin];
    Tally tl;
    for (;;) {
        if (threadIdx.x == 0) s_item = (i32)atomicAdd(&a.next[bin], 1u);
        __syncthreads();
        const i32 item = s_item;
        __syncthreads();
        if ((u32)item >= n) break;
        const i32 x = a.items[item];
        const i64 wx = (i64)a.wi[x];
        int logcap = 6;
        while ((i64(1) << logcap) < 2 * wx && logcap < LOGCAP) ++logcap;
        A.init(logcap, threadIdx.x, BLOCK);
        __syncthreads();
        peel_item<BLOCK>(a, x, A, sm, tl);
    }
    tl.flush(a.kc, a.wedges);
}

// Heavy active vertices: the live Y lists are sorted by X id, so the wedges
// of x whose far end lies in a key tile [r0, r0 + 2^TLOG) form one run of
// every list.  A work item is one (vertex, tile) pair, so the tiles of one
// vertex run on different workgroups at once: each finds the run of every
// neighbour's list by the lockstep search of run_bounds and counts the run's
// wedges in LDS (the last wave claims the next item meanwhile).  A
// count c(x, x') never exceeds the degree of x, so when every degree of the
// graph is below 2^16 (PACK) two 16-bit counters share a word and a tile
// covers 2^16 keys; otherwise each key has a 32-bit counter and a tile
// covers 2^15 keys in the same LDS.  A counter word that leaves zero sets
// its bit in a touched bitmap, and the epilogue visits only the touched
// words, turning counts c >= 2 into updates.  Key tiles are disjoint, so
// every (x, x') pair is completed by exactly one item.  No global atomic is
// issued per wedge.
template <int TLOG, bool PACK>
__global__ __launch_bounds__(512) void k_tip_peel_tiled(PeelArgs a, int bin) {
    constexpr int BLOCK = 512;
    constexpr int KPW = PACK ? 2 : 1;  // keys per counter word
    constexpr int WORDS = (1 << TLOG) / KPW;
    constexpr int BWORDS = WORDS / 32;
    __shared__ u32 cnt[WORDS];
    __shared__ u32 bm[BWORDS];
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_item;
    for (int i = threadIdx.x; i < WORDS; i += BLOCK) cnt[i] = 0;
    for (int i = threadIdx.x; i < BWORDS; i += BLOCK) bm[i] = 0;
    const u64 nt = (u64)a.ntiles;
    const u64 n = (u64)a.nitems[bin] * nt;
    const u64 B = *a.bound;
    Tally tl;
    // the last wave claims the next item while the others start this one
    constexpr int CLAIM = BLOCK - WAVE;
    if (threadIdx.x == CLAIM) s_item = atomicAdd((unsigned long long *)a.tnext, 1ull);
    __syncthreads();
    for (;;) {
        const u64 item = s_item;
        __syncthreads();
        if (item >= n) break;
        if (threadIdx.x == CLAIM) s_item = atomicAdd((unsigned long long *)a.tnext, 1ull);
        const i32 x = a.items[item / nt];
        const u32 t = (u32)(item % nt);
        const i64 r0 = (i64)t << TLOG;
        const i64 r1 = r0 + (i64(1) << TLOG) < a.nx ? r0 + (i64(1) << TLOG) : a.nx;
        const i64 jb = a.xrow[x];
        const i32 d = (i32)(a.xrow[x + 1] - jb);
        if (threadIdx.x == 0 && t == 0) {
            tl.segments += (u64)d;
            tl.items += 1;
        }
        bool any = false;
        for (i32 cb = 0; cb < d; cb += BLOCK) {
            const i32 j = cb + threadIdx.x;
            i32 pl = 0;
            i64 moff = 0;
            if (j < d) {
                const i32 y = a.xadj[jb + j];
                const i64 base = a.yrow[y];
                i64 lo, e;
                run_bounds(a.yadj, base, base + a.ylen[y], a.nx, r0, r1, lo, e);
                pl = (i32)(e - lo);
                moff = lo;
            }
            i32 tot;
            const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
            if (tot == 0) continue;  // block-uniform
            any = true;
            s_pre[threadIdx.x] = incl;
            s_moff[threadIdx.x] = moff;
            __syncthreads();
            const int last = (d - cb < BLOCK ? d - cb : BLOCK) - 1;
            constexpr int UNR = 6;
            for (i32 kb = 0; kb < tot; kb += UNR * BLOCK) {
                i32 xq[UNR];
                run_ends<UNR>(a.yadj, s_pre, s_moff, last, kb + (i32)threadIdx.x * UNR, tot, x, xq);
#pragma unroll
                for (int q = 0; q < UNR; ++q) {
                    const i32 xp = xq[q];
                    if (xp == x) continue;
                    ++tl.wedges;
                    const i32 o = xp - (i32)r0;
                    const u32 wi = PACK ? (u32)o >> 1 : (u32)o;
                    const u32 inc = PACK ? 1u << ((o & 1) << 4) : 1u;
                    if (atomicAdd(&cnt[wi], inc) == 0u) atomicOr(&bm[wi >> 5], 1u << (wi & 31));
                }
            }
            __syncthreads();
        }
        const i32 nbw = any ? (i32)(((r1 - r0 + KPW - 1) / KPW) + 31) >> 5 : 0;
        for (i32 bw = threadIdx.x; bw < nbw; bw += BLOCK) {
            u32 bits = bm[bw];
            if (!bits) continue;
            bm[bw] = 0;
            while (bits) {
                // up to 8 / KPW touched words (eight keys) per batch
                i32 kk[8];
                u32 cc[8];
#pragma unroll
                for (int q = 0; q < 8 / KPW; ++q) {
#pragma unroll
                    for (int h = 0; h < KPW; ++h) {
                        kk[KPW * q + h] = -1;
                        cc[KPW * q + h] = 0;
                    }
                    if (bits) {
                        const i32 wi = bw * 32 + (__ffs(bits) - 1);
                        bits &= bits - 1;
                        const u32 v = cnt[wi];
                        cnt[wi] = 0;
                        if (PACK) {
                            cc[KPW * q] = v & 0xFFFFu;
                            cc[KPW * q + 1] = v >> 16;
                        } else {
                            cc[KPW * q] = v;
                        }
#pragma unroll
                        for (int h = 0; h < KPW; ++h) kk[KPW * q + h] = (i32)r0 + KPW * wi + h;
                    }
                }
                apply_updates<8>(a, B, kk, cc, tl);
            }
        }
        __syncthreads();
    }
    tl.flush(a.kc, a.wedges);
}

// Heavy active vertices whose wedges are many but whose degree is small (a
// few neighbours with long lists, the common case under power-law degrees):
// the wedges of x are cut into R_x = ceil(w_x / H_RANGE_W) ranges of the
// span of X ids in its live lists (the first and last range reach the ends
// of the key space), and one work item is one (vertex, range) pair.  Each range
// counts c(x, x') in an LDS hash table of 2^LOGCAP slots (twice the wedges
// of an item whose keys are spread evenly, and small enough for two
// workgroups per CU); the run of every neighbour list inside the range is
// found by a lockstep search (none when R_x = 1).  An item one of whose keys
// finds its probe sequence full is counted again in HBM (see the kernel), so
// the result is exact for any key skew.
constexpr i64 H_RANGE_W = 4096;
// At most H_RANGE_MAX ranges per vertex: a vertex above H_RANGE_MAX *
// H_RANGE_W wedges has items of more than H_RANGE_W wedges, whose distinct
// keys can still fill the table (its items then take the exact overflow
// pass).  Finer ranges for those vertices cost more in repeated list
// searches than the rare overflow (100M-edge graph: a cap of 256 or 65536
// ranges took the range kernel from 2.66 to 2.93 s).  The cap also shrinks to
// 2^31 / (vertices in the bin), so the item total of a round (32-bit) cannot
// wrap.
constexpr u32 H_RANGE_MAX = 64;
constexpr int H_PROBE = 64;

// R_x of every item of a bin and their exclusive prefix (one workgroup)
__global__ __launch_bounds__(1024) void k_range_split(const i32 *items, const u32 *nbin, int bin, const u64 *wi, u32 *off,
                                                      u32 *total) {
    __shared__ i32 s_wave[1024 / WAVE];
    const u32 n = nbin[bin];
    const u32 rcap0 = 0x80000000u / (n > 0 ? n : 1u);
    const u64 rcap = rcap0 < 1u ? 1u : (rcap0 > H_RANGE_MAX ? H_RANGE_MAX : rcap0);
    u32 carry = 0;
    for (u32 base = 0; base < n; base += 1024) {
        const u32 i = base + threadIdx.x;
        i32 r = 0;
        if (i < n) {
            const u64 w = wi[items[i]];
            const u64 q = (w + (u64)H_RANGE_W - 1) / (u64)H_RANGE_W;
            r = (i32)(q < 1 ? 1 : (q > rcap ? rcap : q));
        }
        i32 tot;
        const i32 incl = block_incl_scan_i32<1024>(r, s_wave, tot);
        if (i < n) off[i] = carry + (u32)(incl - r);
        carry += (u32)tot;
    }
    if (threadIdx.x == 0) {
        off[n] = carry;
        *total = carry;
    }
}

// Item claim of the key-range path, run by one whole wave: the next item
// index, then the vertex that owns it (the last h with off[h] <= item; off
// is strictly increasing with off[nh] = n) by a 64-way search, one probe per
// lane, so a few dependent loads resolve it, then its row and the live list
// of each of its first 64 neighbours.  The result goes to LDS for the next
// iteration, so those dependent loads leave the next item's critical path.
struct RangeItem {
    u32 item;
    i32 x;
    u32 r, R;
    i64 k0, k1;  // the item's key range
    i64 jb;
    i32 d;
    i64 base[WAVE];  // live list of neighbour j < 64: start and length
    i32 len[WAVE];
};

__device__ __forceinline__ void claim_range_item(const PeelArgs &a, int bin, const u32 *off, u32 nh, u32 n, RangeItem *out) {
    const int lane = threadIdx.x & (WAVE - 1);
    u32 it = 0;
    if (lane == 0) it = atomicAdd(&a.next[bin], 1u);
    it = __shfl(it, 0, WAVE);
    if (it < n) {
        u32 lo = 0, hi = nh - 1;
        while (lo < hi) {
            const u32 span = hi - lo;
            const u32 p = lo + (u32)(((u64)(lane + 1) * span + WAVE - 1) / WAVE);
            const int c = __popcll(__ballot(off[p] <= it));
            const u32 nlo = c ? lo + (u32)(((u64)c * span + WAVE - 1) / WAVE) : lo;
            const u32 nhi = c < WAVE ? lo + (u32)(((u64)(c + 1) * span + WAVE - 1) / WAVE) - 1 : hi;
            lo = nlo;
            hi = nhi;
        }
        const i32 x = a.items[lo];
        const i64 jb = a.xrow[x];
        const i32 d = (i32)(a.xrow[x + 1] - jb);
        if (lane < d) {
            const i32 y = a.xadj[jb + lane];
            out->base[lane] = a.yrow[y];
            out->len[lane] = a.ylen[y];
        }
        if (lane == 0) {
            const u32 r = it - off[lo], R = off[lo + 1] - off[lo];
            // the R ranges divide the span of x's 2-hop ids; the first and
            // last reach the ends of the key space, so they cover every key
            i64 klo = a.kspan[2 * (i64)x], span = (i64)a.kspan[2 * (i64)x + 1] - klo + 1;
            if (span <= 0) {
                klo = 0;
                span = a.nx;
            }
            out->x = x;
            out->r = r;
            out->R = R;
            out->k0 = r == 0 ? 0 : klo + (i64)r * span / R;
            out->k1 = r + 1 == R ? a.nx : klo + (i64)(r + 1) * span / R;
            out->jb = jb;
            out->d = d;
        }
    }
    if (lane == 0) out->item = it;
}

template <int LOGCAP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_tip_peel_hrange(PeelArgs a, int bin, const u32 *off, const u32 *total) {
    constexpr u32 CAP = 1u << LOGCAP;
    __shared__ i32 keys[CAP];
    __shared__ u32 vals[CAP];
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u32 s_ntouch, s_ovf, s_set;
    __shared__ RangeItem s_it[2];
    for (u32 i = threadIdx.x; i < CAP; i += BLOCK) {
        keys[i] = -1;
        vals[i] = 0;
    }
    if (threadIdx.x == 0) {
        s_ntouch = 0;
        s_ovf = 0;
    }
    const u32 nh = a.nitems[bin];
    const u32 n = *total;
    const u64 B = *a.bound;
    const int probe = a.hprobe;
    Tally tl;
    // the last wave claims and resolves the next item into the other
    // buffer while the others start this one
    const bool claimer = threadIdx.x >= BLOCK - WAVE;
    int cur = 0;
    if (claimer) claim_range_item(a, bin, off, nh, n, &s_it[0]);
    __syncthreads();
    for (;; cur ^= 1) {
        const RangeItem &ci = s_it[cur];
        const u32 item = ci.item;
        if (item >= n) break;
        if (claimer) claim_range_item(a, bin, off, nh, n, &s_it[cur ^ 1]);
        const i32 x = ci.x;
        const u32 r = ci.r;
        const i64 k0 = ci.k0, k1 = ci.k1;
        const i64 jb = ci.jb;
        const i32 d = ci.d;
        if (threadIdx.x == 0 && r == 0) {
            tl.segments += (u64)d;
            tl.items += 1;
        }
        // Pass 0 counts in the LDS table.  If a key finds its probe
        // sequence full, the item's LDS counts are dropped and pass 1
        // counts the whole item again in one of H_OVF sets of HBM counters
        // that all workgroups share, each under a lock (one item per set at
        // a time; a set's counters are zero between holders), so the result
        // is exact for any key skew.
        bool redo = false;
        u32 *gc = nullptr;
        i32 *gt = nullptr;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                if (!redo) break;  // block-uniform
                if (threadIdx.x == 0) {
                    u32 k = blockIdx.x % H_OVF;
                    while (atomicCAS(&a.dlock[k], 0u, 1u) != 0u) {
                        k = (k + 1) % H_OVF;
                        if (k == blockIdx.x % H_OVF) __builtin_amdgcn_s_sleep(8);
                    }
                    __threadfence();
                    s_set = k;
                }
                __syncthreads();
                gc = a.dcnt + (i64)s_set * a.nx;
                gt = a.dtouch + (i64)s_set * a.nx;
            }
            for (i32 cb = 0; cb < d; cb += BLOCK) {
                const i32 j = cb + threadIdx.x;
                i32 pl = 0;
                i64 moff = 0;
                if (j < d) {
                    i64 base;
                    i32 len;
                    if (j < WAVE) {
                        base = ci.base[j];
                        len = ci.len[j];
                    } else {
                        const i32 y = a.xadj[jb + j];
                        base = a.yrow[y];
                        len = a.ylen[y];
                    }
                    i64 b0, e;
                    run_bounds(a.yadj, base, base + len, a.nx, k0, k1, b0, e);
                    pl = (i32)(e - b0);
                    moff = b0;
                }
                i32 tot;
                const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                if (tot == 0) continue;  // block-uniform
                s_pre[threadIdx.x] = incl;
                s_moff[threadIdx.x] = moff;
                __syncthreads();
                const int last = (d - cb < BLOCK ? d - cb : BLOCK) - 1;
                constexpr int UNR = 8;
                for (i32 kb = 0; kb < tot; kb += UNR * BLOCK) {
                    i32 xq[UNR];
                    run_ends<UNR>(a.yadj, s_pre, s_moff, last, kb + (i32)threadIdx.x * UNR, tot, x, xq);
                    if (pass == 1) {
#pragma unroll
                        for (int q = 0; q < UNR; ++q) {
                            const i32 xp = xq[q];
                            if (xp == x) continue;
                            const u32 old = __hip_atomic_fetch_add(&gc[xp], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if (old == 0) {
                                const u32 t = atomicAdd(&s_ntouch, 1u);
                                __hip_atomic_store(&gt[t], xp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
                        }
                        continue;
                    }
                    // Linear probing over the first `probe` slots.  The first
                    // probe of all UNR keys is one batch of compare-and-swaps
                    // issued together (claim the home slot if empty; a
                    // skipped wedge compares against -2, which no slot holds,
                    // so it writes nothing), so most keys settle after one
                    // LDS round trip shared by the batch; the rest continue
                    // one by one from the next slot.
                    u32 hs[UNR];
                    i32 kk[UNR];
#pragma unroll
                    for (int q = 0; q < UNR; ++q) {
                        hs[q] = hash32((u32)xq[q]) >> (32 - LOGCAP);
                        kk[q] = atomicCAS(&keys[hs[q]], xq[q] != x ? -1 : -2, xq[q]);
                    }
#pragma unroll
                    for (int q = 0; q < UNR; ++q)
                        if (kk[q] == -1) kk[q] = xq[q];
#pragma unroll
                    for (int q = 0; q < UNR; ++q) {
                        const i32 xp = xq[q];
                        if (xp == x) continue;
                        ++tl.wedges;
                        u32 h = hs[q];
                        bool done = kk[q] == xp;
                        for (int p = 1; p < probe && !done; ++p) {
                            h = (h + 1) & (CAP - 1);
                            const i32 k2 = keys[h];
                            if (k2 == xp) {
                                done = true;
                            } else if (k2 == -1) {
                                const i32 prev = atomicCAS(&keys[h], -1, xp);
                                done = prev == -1 || prev == xp;
                            }
                        }
                        if (done)
                            atomicAdd(&vals[h], 1u);
                        else
                            s_ovf = 1;
                    }
                }
                __syncthreads();
            }
            if (pass == 0) {
                // the LDS entries: applied, or dropped when the item overflowed
                redo = s_ovf != 0;
                constexpr int NB = 8;
                for (u32 i0 = threadIdx.x; i0 < CAP; i0 += NB * BLOCK) {
                    i32 kk[NB];
                    u32 cc[NB];
#pragma unroll
                    for (int q = 0; q < NB; ++q) {
                        const u32 i = i0 + q * BLOCK;
                        kk[q] = redo ? -1 : keys[i];
                        cc[q] = vals[i];
                        keys[i] = -1;
                        vals[i] = 0;
                    }
                    apply_updates<NB>(a, B, kk, cc, tl);
                }
                __syncthreads();
                if (threadIdx.x == 0) s_ovf = 0;
            } else {
                // the touched HBM counters, cleared for the next holder
                const u32 nt = s_ntouch;
                for (u32 i0 = threadIdx.x; i0 < nt; i0 += 4 * BLOCK) {
                    i32 kk[4];
                    u32 cc[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const u32 i = i0 + q * BLOCK;
                        kk[q] = i < nt ? __hip_atomic_load(&gt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
                        cc[q] = kk[q] >= 0 ? __hip_atomic_exchange(&gc[kk[q]], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                           : 0u;
                    }
                    apply_updates<4>(a, B, kk, cc, tl);
                }
                __threadfence();
                __syncthreads();
                if (threadIdx.x == 0) {
                    s_ntouch = 0;
                    atomicExch(&a.dlock[s_set], 0u);
                }
            }
        }
    }
    tl.flush(a.kc, a.wedges);
}

// Active vertices with few neighbours: C(c, 2) for a vertex x' is the number
// of pairs {y_i, y_j} of x's neighbours whose live lists both hold x', so the
// decrements come from the pairwise intersections of x's neighbour lists:
// every element of the shorter list of a pair is searched in the longer one
// (both sorted by X id) and each hit on an alive vertex lowers its support by
// one.  The total per vertex equals the wedge-counting path's C(c, 2).  One
// wave per vertex.
__global__ void k_tip_peel_pairs(PeelArgs a, int bin) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = a.nitems[bin];
    const i32 *items = a.items;
    Tally tl;
    for (i64 it = wave; it < n; it += nwaves) {
        const i32 x = items[it];
        const i64 jb = a.xrow[x];
        const int d = (int)(a.xrow[x + 1] - jb);
        // neighbour lists in lanes 0..d-1
        i64 lb = 0;
        i32 ll = 0;
        if (lane < d) {
            const i32 y = a.xadj[jb + lane];
            lb = a.yrow[y];
            ll = a.ylen[y];
        }
        if (lane == 0) {
            tl.segments += (u64)d;
            tl.items += 1;
        }
        for (int i = 0; i < d; ++i) {
            const i64 bi = __shfl(lb, i, WAVE);
            const i32 li = __shfl(ll, i, WAVE);
            for (int j = i + 1; j < d; ++j) {
                const i64 bj = __shfl(lb, j, WAVE);
                const i32 lj = __shfl(ll, j, WAVE);
                const bool si = li <= lj;
                const i64 sb = si ? bi : bj, gb = si ? bj : bi;
                const i32 sl = si ? li : lj, gl = si ? lj : li;
                for (i32 k = lane; k < sl; k += WAVE) {
                    const i32 v = a.yadj[sb + k];
                    ++tl.wedges;
                    if (v == x) continue;
                    // lower bound of v in the longer list
                    i32 lo = 0, hi = gl;
                    while (lo < hi) {
                        const i32 md = (lo + hi) >> 1;
                        if (a.yadj[gb + md] < v) lo = md + 1; else hi = md;
                    }
                    if (lo == gl || a.yadj[gb + lo] != v) continue;
                    if (a.st[v] != ST_ALIVE) continue;
                    atomicAdd((unsigned long long *)&a.sup[v], (unsigned long long)(0ull - 1ull));
                    ++tl.atomics;
                }
            }
        }
    }
    tl.flush(a.kc, a.wedges);
}

// ------------------------------------------------------------------ CD helpers

// Wedges of each active vertex over the live lists (one wave per vertex),
// their total (the batch rule's wedge count of the active set, Section 5.1),
// and the work bins: small / medium LDS hash, key ranges, key tiles, pairs.
// A vertex of the key-range bin also gets the span [lo, hi] of the X ids in
// its live lists, which its ranges divide: ids need not spread over the
// whole key space (in a disjoint union of graphs every vertex's 2-hop ids lie
// in its own graph's id block).
__global__ void k_item_work(const i32 *F, const u32 *nF, const i64 *xrow, const i32 *xadj, const i64 *yrow,
                            const i32 *yadj, const i32 *ylen, u64 *wi, u64 *wsum, i32 *lists, i64 stride, u32 *nbin,
                            u64 huge_w, i32 *kspan) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *nF;
    for (i64 i = wave; i < n; i += nwaves) {
        const i32 x = F[i];
        const i64 jb = xrow[x], je = xrow[x + 1];
        u64 s = 0;
        for (i64 j = jb + lane; j < je; j += WAVE) s += (u64)ylen[xadj[j]];
        for (int dd = WAVE / 2; dd > 0; dd >>= 1) s += __shfl_down(s, dd, WAVE);
        const i64 d = je - jb;
        // a vertex with one neighbour shares at most one with anyone: c <= 1,
        // C(c, 2) = 0, so peeling it updates nothing and it is not walked
        if (d < 2) s = 0;
        // few neighbours: cost of the pairwise list intersections (each
        // element of the shorter list searched in the longer one)
        u64 pc = ~0ull;
        if (d >= 2 && d <= PAIR_DMAX) {
            const u32 l = lane < d ? (u32)ylen[xadj[jb + lane]] : 0u;
            u64 acc = 0;
            for (int i = 0; i < (int)d; ++i) {
                const u32 li = __shfl(l, i, WAVE);
                if (lane > i && lane < d) {
                    const u32 mn = li < l ? li : l, mx = li < l ? l : li;
                    acc += (u64)mn * (u64)(bits_of(mx) + 1);
                }
            }
            for (int dd = WAVE / 2; dd > 0; dd >>= 1) acc += __shfl_down(acc, dd, WAVE);
            pc = acc;
        }
        int b = -1;
        if (lane == 0) {
            const bool pairs = s >= 2 && pc != ~0ull && PAIR_COST * pc < s;
            // the work estimate is what the chosen method walks
            const u64 sw = pairs ? pc : s;
            wi[x] = sw;
            atomicAdd((unsigned long long *)wsum, (unsigned long long)sw);
            if (s >= 2) {
                if (pairs) b = 4;
                else if (s <= (u64)T_SMALL_W) b = 0;
                else if (s <= (u64)T_MEDIUM_W) b = 1;
                else if (s <= huge_w) b = 2;
                else b = 3;
                u32 p = atomicAdd(&nbin[b], 1u);
                lists[b * stride + p] = x;
            }
        }
        b = __shfl(b, 0, WAVE);
        if (b == 2) {
            i32 lo = 0x7fffffff, hi = -1;
            for (i64 j = jb + lane; j < je; j += WAVE) {
                const i32 y = xadj[j];
                const i32 l = ylen[y];
                if (l > 0) {
                    const i64 yb = yrow[y];
                    const i32 h0 = yadj[yb], t0 = yadj[yb + l - 1];
                    lo = h0 < lo ? h0 : lo;
                    hi = t0 > hi ? t0 : hi;
                }
            }
            for (int dd = WAVE / 2; dd > 0; dd >>= 1) {
                const i32 ol = __shfl_xor(lo, dd, WAVE), oh = __shfl_xor(hi, dd, WAVE);
                lo = ol < lo ? ol : lo;
                hi = oh > hi ? oh : hi;
            }
            if (lane == 0) {
                kspan[2 * (i64)x] = lo;
                kspan[2 * (i64)x + 1] = hi;
            }
        }
    }
}

// w_x = sum of live Y degrees over N_x, one wave per row
__global__ void k_work_full(const i64 *xrow, const i32 *xadj, const i32 *ydeg, const unsigned char *st, i64 nx, u64 *w) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    for (i64 x = wave; x < nx; x += nwaves) {
        if (st && st[x] != ST_ALIVE) continue;
        u64 s = 0;
        for (i64 j = xrow[x] + lane; j < xrow[x + 1]; j += WAVE) s += (u64)ydeg[xadj[j]];
        for (int d = WAVE / 2; d > 0; d >>= 1) s += __shfl_down(s, d, WAVE);
        if (lane == 0) w[x] = s;
    }
}

// Snapshot of the partition start (initialisation vector) and the first
// active set: alive x with support below the bound.
__global__ void k_frontier(unsigned char *st, const u64 *sup, const u64 *w, u64 *init, u64 *wsnap, i32 *part, i64 nx,
                           TipCtl *ctl, i32 pid, int snapshot, i32 *F) {
    const u64 B = ctl->bound;
    const i64 stride = (i64)gridDim.x * blockDim.x;
    const i64 nn = (nx + WAVE - 1) / WAVE * WAVE;  // wave-uniform trip count
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nn; x += stride) {
        bool take = false;
        if (x < nx && st[x] == ST_ALIVE) {
            const u64 s = sup[x];
            if (snapshot) {
                init[x] = s;
                wsnap[x] = w[x];
            }
            take = s < B;
        }
        const u32 p = wave_append(&ctl->nF, take);
        if (take) {
            st[x] = ST_ACTIVE;
            part[x] = pid;
            F[p] = (i32)x;
        }
    }
}

// Active vertices become peeled: their Y neighbours lose one live degree and
// are queued for list compaction (one queue append per wave and step).  One
// wave per vertex.
__global__ void k_retire(const i32 *F, const u32 *nF, const i64 *xrow, const i32 *xadj, unsigned char *st, i32 *ydeg,
                         unsigned char *ydirty, i32 *dirty, u32 *ndirty, int dynamic) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *nF;
    for (i64 i = wave; i < n; i += nwaves) {
        const i32 x = F[i];
        if (lane == 0) st[x] = ST_PEELED;
        const i64 je = xrow[x + 1];
        for (i64 j0 = xrow[x]; j0 < je; j0 += WAVE) {  // wave-uniform trip count
            const i64 j = j0 + lane;
            bool fresh = false;
            i32 y = 0;
            if (j < je) {
                y = xadj[j];
                atomicSub(&ydeg[y], 1);
                if (dynamic) {
                    // byte flag per y: first setter queues y
                    unsigned int *word = (unsigned int *)(ydirty + (y & ~3));
                    const unsigned int bit = 0xFFu << (8 * (y & 3));
                    fresh = (atomicOr(word, bit) & bit) == 0;
                }
            }
            const u32 p = wave_append(ndirty, fresh);
            if (fresh) dirty[p] = y;
        }
    }
}

// Work of the partition's vertices (all peeled by now), summed for the
// scaling factor of the next partition; one device atomic per workgroup.
__global__ __launch_bounds__(256) void k_part_work(const unsigned char *st, const i32 *part, const u64 *wsnap, i64 nx,
                                                   i32 pid, TipCtl *ctl) {
    __shared__ u64 red[256 / WAVE];
    u64 t = 0;
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x)
        if (st[x] == ST_PEELED && part[x] == pid) t += wsnap[x];
    t = block_sum_u64<256>(t, red);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)&ctl->est_final, (unsigned long long)t);
}

__global__ void k_activate(const i32 *F2, const u32 *nF2, unsigned char *st, i32 *part, const TipCtl *ctl) {
    const u32 n = *nF2;
    const i32 pid = ctl->pid;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        i32 x = F2[i];
        st[x] = ST_ACTIVE;
        part[x] = pid;
    }
}

// In-place compaction of dirty Y lists to their alive entries; one wave per
// list, four 64-entry chunks per step (their loads in flight together) with
// a ballot prefix.
__global__ void k_compact(const i32 *dirty, const u32 *ndirty, const i64 *yrow, i32 *yadj, i32 *ylen,
                          unsigned char *ydirty, const unsigned char *st) {
    constexpr int CU = 4;
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *ndirty;
    const u64 lt = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    for (i64 i = wave; i < n; i += nwaves) {
        i32 y = dirty[i];
        const i64 b = yrow[y];
        const i32 len = ylen[y];
        i32 out = 0;
        for (i32 k0 = 0; k0 < len; k0 += CU * WAVE) {
            i32 xv[CU];
#pragma unroll
            for (int c = 0; c < CU; ++c) {
                const i32 k = k0 + c * WAVE + lane;
                xv[c] = k < len ? yadj[b + k] : -1;
            }
            bool keep[CU];
#pragma unroll
            for (int c = 0; c < CU; ++c) keep[c] = xv[c] >= 0 && st[xv[c]] == ST_ALIVE;
#pragma unroll
            for (int c = 0; c < CU; ++c) {
                const u64 bal = __ballot(keep[c]);
                if (keep[c]) yadj[b + out + __popcll(bal & lt)] = xv[c];
                out += __popcll(bal);
            }
        }
        if (lane == 0) {
            ylen[y] = out;
            ydirty[y] = 0;
        }
    }
}

// A partition whose range is a single support value k (its bound is the
// smallest alive support k plus one): every vertex it peels has tip number k
// (the running maximum of the bottom-up order is k while the cascade below
// k + 1 runs), so it needs no fine-grained peeling; its level is recorded.
__global__ void k_level_bound(TipCtl *ctl, const u64 *mn, u64 *plev) {
    ctl->s = mn[0];
    *plev = mn[0];
}

// Work estimate summed over the alive vertices (one device atomic per block).
__global__ __launch_bounds__(256) void k_alive_work(const unsigned char *st, const u64 *w, i64 nx, u64 *out) {
    __shared__ u64 red[256 / WAVE];
    u64 t = 0;
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x)
        if (st[x] == ST_ALIVE) t += w[x];
    t = block_sum_u64<256>(t, red);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)out, (unsigned long long)t);
}

// the learned bound never falls to or below the smallest alive support
__global__ void k_learned_guard(TipCtl *ctl, const u64 *mn) {
    if (ctl->s < mn[0]) ctl->s = mn[0];
}

__global__ void k_set_bound(TipCtl *ctl, int last, i32 pid) {
    ctl->bound = last ? ~0ull : ctl->s + 1;
    ctl->pid = pid;
    ctl->nF = 0;
    ctl->nF2 = 0;
    ctl->wF = 0;
    ctl->est_final = 0;
    for (int b = 0; b < 5; ++b) ctl->nbin[b] = ctl->next[b] = 0;
    ctl->tnext = 0;
}

__global__ void k_record_bound(const TipCtl *ctl, u64 *out) { *out = ctl->bound; }

// Start of a captured round: an empty active set makes the round a no-op
// (every kernel finds nothing to do).  An active set holding every alive
// vertex needs no updates, and one whose wedges exceed the recount bound is
// handed to a recount after the replay (Section 5.1): both empty the work
// bins so the round only retires the set.
__global__ void k_round_begin(TipCtl *ctl, int batch) {
    const u32 nF = ctl->nF;
    if (nF == 0) return;
    ctl->rounds += 1;
    const bool all = (u64)nF == ctl->alive;
    const bool rec = !all && batch && ctl->wF > ctl->wbound;
    if (all || rec)
        for (int b = 0; b < 5; ++b) ctl->nbin[b] = 0;
    if (rec) ctl->recount = 1;
    ctl->alive -= nF;
}

__global__ void k_next_round(TipCtl *ctl) {
    // next active set becomes current; counters of the round are cleared
    ctl->nF = ctl->nF2;
    ctl->nF2 = 0;
    ctl->wF = 0;
    for (int b = 0; b < 5; ++b) ctl->nbin[b] = ctl->next[b] = 0;
    ctl->tnext = 0;
    ctl->ndirty = 0;
}

__global__ void k_scale(TipCtl *ctl) {
    // s_{i+1} = initial estimate / final estimate of partition i
    double fin = (double)ctl->est_final;
    ctl->scale = fin > 0 ? (double)ctl->est_init / fin : 1.0;
    if (!(ctl->scale > 0)) ctl->scale = 1.0;
}

__global__ void k_alive_label(const unsigned char *st, const i32 *gid, i64 n, i64 xoff, i64 nx, unsigned char *alive) {
    for (i64 l = blockIdx.x * (i64)blockDim.x + threadIdx.x; l < n; l += (i64)gridDim.x * blockDim.x) {
        i64 g = gid[l] - xoff;
        alive[l] = (g >= 0 && g < nx) ? (st[g] == ST_ALIVE) : 1;
    }
}

__global__ void k_from_label(const u64 *sup_label, const i32 *label, i64 xoff, i64 nx, const unsigned char *st, u64 *sup) {
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x)
        if (st[x] == ST_ALIVE) sup[x] = sup_label[label[x + xoff]];
}

__global__ void k_min_deg_sum(const i64 *xrow, const i32 *xadj, const i32 *ydeg, i64 nx, u64 *out) {
    // sum over edges of min(d_x, d_y): the wedge bound of one counting pass
    u64 s = 0;
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x) {
        i64 dx = xrow[x + 1] - xrow[x];
        for (i64 j = xrow[x]; j < xrow[x + 1]; ++j) {
            i64 dy = ydeg[xadj[j]];
            s += (u64)(dx < dy ? dx : dy);
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) s += __shfl_down(s, d, WAVE);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)out, (unsigned long long)s);
}

__global__ void k_degrees_y(const i64 *yrow, i64 ny, i32 *ydeg, i32 *ylen) {
    for (i64 y = blockIdx.x * (i64)blockDim.x + threadIdx.x; y < ny; y += (i64)gridDim.x * blockDim.x) {
        i32 d = (i32)(yrow[y + 1] - yrow[y]);
        ydeg[y] = d;
        ylen[y] = d;
    }
}

// Smallest and largest alive support (grid-stride, one atomic pair per
// wave; launched with a capped grid so the two counters see few atomics).
// Seeded random bounds (schedule-invariance tests) draw theta(i+1) between
// them; single levels and the learned guard use the smallest.
__global__ void k_random_bound(const u64 *sup, const unsigned char *st, i64 nx, u64 *mn, u64 *mx) {
    u64 a = ~0ull, b = 0;
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x) {
        if (st[x] != ST_ALIVE) continue;
        u64 s = sup[x];
        a = s < a ? s : a;
        b = s > b ? s : b;
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        u64 o = __shfl_down(a, d, WAVE);
        a = o < a ? o : a;
        o = __shfl_down(b, d, WAVE);
        b = o > b ? o : b;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin((unsigned long long *)mn, (unsigned long long)a);
        atomicMax((unsigned long long *)mx, (unsigned long long)b);
    }
}

__device__ inline u64 splitmix64(u64 z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_random_pick(TipCtl *ctl, const u64 *mn, const u64 *mx, u64 seed, int i) {
    u64 lo = *mn, hi = *mx;
    u64 span = hi - lo + 1;
    u64 r = splitmix64(seed * 1000003ull + (u64)i);
    // bias toward small steps so that several partitions form
    u64 step = span > 1 ? r % (span / 4 + 1) : 0;
    ctl->s = lo + step;
}

// ------------------------------------------------------------------ FD

struct FdArgs {
    const i64 *xrow;
    const i32 *xadj;
    const i32 *xs;       // X ids grouped by partition
    const i64 *poff;     // [np+1]
    const i32 *loc;      // position of x inside its partition
    const i32 *yps;      // Y lists grouped by partition
    const i64 *flo;      // per X-CSR entry: start of N_y restricted to p(x)
    const i32 *flen;     // per X-CSR entry: its length
    const i32 *queue;    // partitions, decreasing work
    i32 np;
    u32 *head;
    const u64 *init;
    const u64 *plev;     // level of a single-value partition, ~0 otherwise
    u64 *theta;
    // per-workgroup scratch, stride maxni
    u64 *lsup;
    unsigned char *lst;
    u32 *lcnt;
    i32 *ltouch;
    i32 *lbatch;
    i32 *lheavy;
    i64 maxni;
    i32 pack16;          // every degree below 2^16: packed 16-bit LDS counters allowed
    u64 *wedges;
    KCounters *kc;
};

// One workgroup peels one partition at a time with bottom-up peeling on its
// induced subgraph, a whole level at once: take every alive vertex at the
// current minimum support k, lower every other alive vertex's support by
// C(c, 2) for each of them (c = common neighbours inside the partition), then
// clamp to k.  The clamps of one level commute, max(k, max(k, s - a) - b) =
// max(k, s - a - b), so the decrements are applied in any order as signed
// atomic subtractions and the clamp is taken once at the end of the level.
// Batch vertices with at most FD_WAVE_W wedges inside the partition are
// counted one per wave in a private LDS hash; the rest one at a time by the
// whole workgroup with the partition-wide counters.
constexpr int FD_BLOCK = 512;
constexpr int FD_LDS_NI = 4096;  // partitions this small live in LDS
constexpr int FD_WAVE_LOG = 9;                        // per-wave hash slots (log2)
constexpr int FD_WAVE_W = (1 << FD_WAVE_LOG) * 5 / 8;  // wedges a wave hash takes
constexpr int FD_UNR = 4;                              // wedges per lane and step

__global__ __launch_bounds__(FD_BLOCK) void k_tip_fd(FdArgs a) {
    constexpr int BLOCK = FD_BLOCK;
    constexpr int NW = BLOCK / WAVE;
    constexpr int HCAP = 1 << FD_WAVE_LOG;
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ i32 s_wave[NW];
    __shared__ u64 s_red[NW];
    __shared__ i32 s_item;
    __shared__ u32 s_cnt[3];
    // per-wave hashes (keys, then counts); during the heavy phase the same
    // words hold dense packed 16-bit counters over the partition's vertices
    __shared__ u32 hmem[2 * NW * HCAP];
    i32(*hkeys)[HCAP] = reinterpret_cast<i32(*)[HCAP]>(hmem);
    u32(*hvals)[HCAP] = reinterpret_cast<u32(*)[HCAP]>(hmem + NW * HCAP);
    constexpr i32 DENSE_NI = 2 * 2 * NW * HCAP;  // vertices the dense counters cover
    // a partition of at most FD_LDS_NI vertices keeps its supports, states and
    // level batch in LDS; larger ones use the workgroup's HBM slices
    __shared__ i64 s_lsup[FD_LDS_NI];
    __shared__ unsigned char s_lst[FD_LDS_NI];
    __shared__ i32 s_lbatch[FD_LDS_NI];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    i64 *const g_lsup = reinterpret_cast<i64 *>(a.lsup) + blockIdx.x * a.maxni;
    unsigned char *const g_lst = a.lst + blockIdx.x * a.maxni;
    u32 *lcnt = a.lcnt + blockIdx.x * a.maxni;
    i32 *ltouch = a.ltouch + blockIdx.x * a.maxni;
    i32 *const g_lbatch = a.lbatch + blockIdx.x * a.maxni;
    i32 *lheavy = a.lheavy + blockIdx.x * a.maxni;
    for (int i = lane; i < HCAP; i += WAVE) {
        hkeys[wid][i] = -1;
        hvals[wid][i] = 0;
    }
    u64 wedges = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = (i32)atomicAdd(a.head, 1u);
        __syncthreads();
        const i32 qi = s_item;
        __syncthreads();
        if (qi >= a.np) break;
        const i32 pid = a.queue[qi];
        const i64 base = a.poff[pid];
        const i32 ni = (i32)(a.poff[pid + 1] - base);
        const u64 lev = a.plev[pid];
        if (lev != ~0ull) {
            // single-value range: every tip number is its level
            for (i32 k = threadIdx.x; k < ni; k += BLOCK) a.theta[a.xs[base + k]] = lev;
            continue;
        }
        const bool in_lds = ni <= FD_LDS_NI;
        i64 *const lsup = in_lds ? s_lsup : g_lsup;
        unsigned char *const lst = in_lds ? s_lst : g_lst;
        i32 *const lbatch = in_lds ? s_lbatch : g_lbatch;
        // Thread t owns vertices t, t + BLOCK, ...  Each pass that computes
        // a level's minimum also records, in a bit mask, which of the
        // thread's vertices hold the thread's minimum, so the next level's
        // batch comes from the mask instead of another scan (partitions of
        // at most 64 * BLOCK vertices; larger ones scan).
        const bool masked = ni <= 64 * BLOCK;
        u64 mn = ~0ull, cm = 0;
        for (i32 k = threadIdx.x, e = 0; k < ni; k += BLOCK, ++e) {
            const u64 v0 = a.init[a.xs[base + k]];
            st_coherent(&lsup[k], (i64)v0);
            st_coherent(&lst[k], (unsigned char)1);
            st_coherent(&lcnt[k], 0u);
            if (v0 < mn) {
                mn = v0;
                cm = 0;
            }
            if (v0 == mn && e < 64) cm |= 1ull << e;
        }
        u64 kmin = block_min_u64<BLOCK>(mn, s_red);
        __syncthreads();
        i32 remaining = ni;
        while (remaining > 0) {
            if (threadIdx.x == 0) s_cnt[0] = s_cnt[2] = 0;
            __syncthreads();
            if (masked) {
                u64 bits = mn == kmin ? cm : 0ull;
                while (bits) {
                    const i32 k = threadIdx.x + (__ffsll((unsigned long long)bits) - 1) * BLOCK;
                    bits &= bits - 1;
                    const u32 p = atomicAdd(&s_cnt[0], 1u);
                    st_coherent(&lbatch[p], k);
                    st_coherent(&lst[k], (unsigned char)2);
                    a.theta[a.xs[base + k]] = kmin;
                }
            } else {
                for (i32 k = threadIdx.x; k < ni; k += BLOCK) {
                    if (ld_coherent(&lst[k]) == 1 && (u64)ld_coherent(&lsup[k]) == kmin) {
                        const u32 p = atomicAdd(&s_cnt[0], 1u);
                        st_coherent(&lbatch[p], k);
                        st_coherent(&lst[k], (unsigned char)2);
                        a.theta[a.xs[base + k]] = kmin;
                    }
                }
            }
            __syncthreads();
            const i32 nb = (i32)s_cnt[0];
            // wave per batch vertex: count c(x, x') in the wave's hash
            for (i32 b = wid; b < nb; b += NW) {
                const i32 x = a.xs[base + ld_coherent(&lbatch[b])];
                const i64 jb = a.xrow[x], je = a.xrow[x + 1];
                i64 tw = 0;
                for (i64 j = jb + lane; j < je; j += WAVE) tw += a.flen[j];
                for (int d = WAVE / 2; d > 0; d >>= 1) tw += __shfl_xor(tw, d, WAVE);
                if (tw > FD_WAVE_W) {
                    if (lane == 0) lheavy[atomicAdd(&s_cnt[2], 1u)] = x;
                    continue;
                }
                if (tw == 0) continue;
                for (i64 cb = jb; cb < je; cb += WAVE) {
                    const i64 j = cb + lane;
                    i32 pl = 0;
                    i64 moff = 0;
                    if (j < je) {
                        pl = a.flen[j];
                        moff = a.flo[j];
                    }
                    i32 incl = pl;
                    for (int d = 1; d < WAVE; d <<= 1) {
                        const i32 y = __shfl_up(incl, d, WAVE);
                        if (lane >= d) incl += y;
                    }
                    const i32 tot = __shfl(incl, WAVE - 1, WAVE);
                    // lanes walk the wedges of the chunk; the owning entry of
                    // wedge k is the first lane whose inclusive prefix exceeds k
                    s_pre[threadIdx.x] = incl;
                    s_moff[threadIdx.x] = moff;
                    __builtin_amdgcn_wave_barrier();
                    for (i32 kb = 0; kb < tot; kb += FD_UNR * WAVE) {
                      // far ends, local indices and states of FD_UNR wedges
                      // are loaded together (every index is inside the
                      // partition: x itself stands in for wedges past tot)
                      i32 xq[FD_UNR], kq[FD_UNR];
                      unsigned char sq[FD_UNR];
                      run_ends<FD_UNR>(a.yps, s_pre + wid * WAVE, s_moff + wid * WAVE, WAVE - 1, kb + lane * FD_UNR, tot, x,
                                       xq);
#pragma unroll
                      for (int q = 0; q < FD_UNR; ++q) kq[q] = a.loc[xq[q]];
#pragma unroll
                      for (int q = 0; q < FD_UNR; ++q) sq[q] = ld_coherent(&lst[kq[q]]);
#pragma unroll
                      for (int q = 0; q < FD_UNR; ++q) {
                        if (xq[q] == x) continue;
                        ++wedges;
                        const i32 kp = kq[q];
                        if (sq[q] != 1) continue;
                        u32 h = hash32((u32)kp) >> (32 - FD_WAVE_LOG);
                        for (;;) {
                            const i32 kk = hkeys[wid][h];
                            if (kk == kp) break;
                            if (kk == -1) {
                                const i32 prev = atomicCAS(&hkeys[wid][h], -1, kp);
                                if (prev == -1 || prev == kp) break;
                            }
                            h = (h + 1) & (HCAP - 1);
                        }
                        atomicAdd(&hvals[wid][h], 1u);
                      }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                __builtin_amdgcn_wave_barrier();
                for (int i = lane; i < HCAP; i += WAVE) {
                    const i32 kk = hkeys[wid][i];
                    if (kk == -1) continue;
                    const u64 cc = hvals[wid][i];
                    hkeys[wid][i] = -1;
                    hvals[wid][i] = 0;
                    if (cc >= 2) atomicAdd((unsigned long long *)&lsup[kk], (unsigned long long)(0ull - cc * (cc - 1) / 2));
                }
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            // vertices with many wedges: the whole workgroup, one at a time
            const i32 nh = (i32)s_cnt[2];
            // packed 16-bit counters hold c(x, x') <= degree of x < 2^16
            const bool dense = ni <= DENSE_NI && a.pack16;
            if (nh > 0 && dense)
                for (i32 i = threadIdx.x; i < 2 * NW * HCAP; i += BLOCK) hmem[i] = 0;
            __syncthreads();
            for (i32 b = 0; dense && b < nh; ++b) {
                const i32 x = ld_coherent(&lheavy[b]);
                const i64 jb = a.xrow[x], je = a.xrow[x + 1];
                for (i64 cb = jb; cb < je; cb += BLOCK) {
                    const i64 j = cb + threadIdx.x;
                    i32 pl = 0;
                    i64 moff = 0;
                    if (j < je) {
                        pl = a.flen[j];
                        moff = a.flo[j];
                    }
                    i32 tot;
                    const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                    s_pre[threadIdx.x] = incl;
                    s_moff[threadIdx.x] = moff;
                    __syncthreads();
                    const int last = (je - cb < BLOCK ? (int)(je - cb) : BLOCK) - 1;
                    for (i32 kb = 0; kb < tot; kb += FD_UNR * BLOCK) {
                        i32 xq[FD_UNR], kq[FD_UNR];
                        unsigned char sq[FD_UNR];
                        run_ends<FD_UNR>(a.yps, s_pre, s_moff, last, kb + (i32)threadIdx.x * FD_UNR, tot, x, xq);
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) kq[q] = a.loc[xq[q]];
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) sq[q] = ld_coherent(&lst[kq[q]]);
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) {
                            if (xq[q] == x) continue;
                            ++wedges;
                            if (sq[q] != 1) continue;
                            atomicAdd(&hmem[kq[q] >> 1], 1u << ((kq[q] & 1) << 4));
                        }
                    }
                    __syncthreads();
                }
                const i32 nw = (ni + 1) >> 1;
                for (i32 w = threadIdx.x; w < nw; w += BLOCK) {
                    const u32 v = hmem[w];
                    if (!v) continue;
                    hmem[w] = 0;
                    const u64 c0 = v & 0xFFFFu, c1 = v >> 16;
                    if (c0 >= 2) atomicAdd((unsigned long long *)&lsup[2 * w], (unsigned long long)(0ull - c0 * (c0 - 1) / 2));
                    if (c1 >= 2)
                        atomicAdd((unsigned long long *)&lsup[2 * w + 1], (unsigned long long)(0ull - c1 * (c1 - 1) / 2));
                }
                __syncthreads();
            }
            if (nh > 0 && dense) {
                // back to empty wave hashes
                for (i32 i = threadIdx.x; i < NW * HCAP; i += BLOCK) hmem[i] = 0xFFFFFFFFu;
                __syncthreads();
            }
            for (i32 b = 0; !dense && b < nh; ++b) {
                const i32 x = ld_coherent(&lheavy[b]);
                if (threadIdx.x == 0) s_cnt[1] = 0;
                __syncthreads();
                const i64 jb = a.xrow[x], je = a.xrow[x + 1];
                for (i64 cb = jb; cb < je; cb += BLOCK) {
                    const i64 j = cb + threadIdx.x;
                    i32 pl = 0;
                    i64 moff = 0;
                    if (j < je) {
                        pl = a.flen[j];
                        moff = a.flo[j];
                    }
                    i32 tot;
                    const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                    s_pre[threadIdx.x] = incl;
                    s_moff[threadIdx.x] = moff;
                    __syncthreads();
                    const int last = (je - cb < BLOCK ? (int)(je - cb) : BLOCK) - 1;
                    for (i32 kb = 0; kb < tot; kb += FD_UNR * BLOCK) {
                        i32 xq[FD_UNR], kq[FD_UNR];
                        unsigned char sq[FD_UNR];
                        run_ends<FD_UNR>(a.yps, s_pre, s_moff, last, kb + (i32)threadIdx.x * FD_UNR, tot, x, xq);
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) kq[q] = a.loc[xq[q]];
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) sq[q] = ld_coherent(&lst[kq[q]]);
#pragma unroll
                        for (int q = 0; q < FD_UNR; ++q) {
                            if (xq[q] == x) continue;
                            ++wedges;
                            if (sq[q] != 1) continue;
                            const i32 kp = kq[q];
                            if (atomicAdd(&lcnt[kp], 1u) == 0) {
                                const u32 t = atomicAdd(&s_cnt[1], 1u);
                                st_coherent(&ltouch[t], kp);
                            }
                        }
                    }
                    __syncthreads();
                }
                const u32 nt = s_cnt[1];
                for (u32 t = threadIdx.x; t < nt; t += BLOCK) {
                    const i32 kp = ld_coherent(&ltouch[t]);
                    const u64 cc = atomicExch(&lcnt[kp], 0u);
                    if (cc >= 2) atomicAdd((unsigned long long *)&lsup[kp], (unsigned long long)(0ull - cc * (cc - 1) / 2));
                }
                __syncthreads();
            }
            // clamp at the level, retire the batch and find the next level;
            // eight vertices per step with their state and support loads in
            // flight together
            mn = ~0ull;
            cm = 0;
            for (i32 k0 = threadIdx.x, e0 = 0; k0 < ni; k0 += 8 * BLOCK, e0 += 8) {
                unsigned char sv[8];
                i64 vv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const i32 k = k0 + q * BLOCK;
                    sv[q] = ld_coherent(&lst[k < ni ? k : 0]);
                    vv[q] = ld_coherent(&lsup[k < ni ? k : 0]);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const i32 k = k0 + q * BLOCK;
                    if (k >= ni) continue;
                    if (sv[q] == 2) {
                        st_coherent(&lst[k], (unsigned char)0);
                    } else if (sv[q] == 1) {
                        i64 v = vv[q];
                        if (v < (i64)kmin) {
                            v = (i64)kmin;
                            st_coherent(&lsup[k], v);
                        }
                        if ((u64)v < mn) {
                            mn = (u64)v;
                            cm = 0;
                        }
                        if ((u64)v == mn && e0 + q < 64) cm |= 1ull << (e0 + q);
                    }
                }
            }
            remaining -= nb;
            kmin = block_min_u64<BLOCK>(mn, s_red);
            __syncthreads();
        }
    }
    Tally tl;
    tl.wedges = wedges;
    tl.flush(a.kc, a.wedges);
}

// ---- FD preparation kernels

__global__ void k_part_keys(const i32 *part, i64 nx, u64 *keys, i32 *vals) {
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x) {
        keys[x] = (u64)part[x];
        vals[x] = (i32)x;
    }
}

__global__ void k_u32_to_i64_t(const u32 *a, i64 n, i64 *b) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) b[i] = a[i];
}

__global__ void k_loc(const i32 *xs, const i32 *part, const i64 *poff, i64 nx, i32 *loc) {
    for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nx; k += (i64)gridDim.x * blockDim.x) {
        i32 x = xs[k];
        loc[x] = (i32)(k - poff[part[x]]);
    }
}

__device__ inline i64 row_of_t(const i64 *row, i64 n, i64 e) {
    i64 a = 0, b = n;
    while (a < b) {
        i64 c = (a + b + 1) >> 1;
        if (row[c] <= e) a = c; else b = c - 1;
    }
    return a;
}

__global__ void k_ypart_keys(const i64 *yrow, const i32 *yadj_orig, const i32 *part, i64 ny, i64 m, i32 np, u64 *keys, i32 *vals) {
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        i64 y = row_of_t(yrow, ny, e);
        i32 x = yadj_orig[e];
        keys[e] = (u64)y * (u64)np + (u64)part[x];
        vals[e] = x;
    }
}

// For X-CSR entry (x, y): the run of N_y (grouped by partition) whose
// vertices share x's partition; work_p += its length - 1.
__global__ __launch_bounds__(256) void k_fd_segments(const i64 *xrow, const i32 *xadj, i64 nx, i64 mx, const i64 *yrow,
                                                     const i32 *yps, const i32 *part, i64 *flo, i32 *flen, u64 *work,
                                                     i32 np) {
    // per-partition work summed in LDS first when the partitions fit
    constexpr int HB = 2048;
    __shared__ unsigned long long h[HB];
    const bool priv = np <= HB;
    if (priv) {
        for (int b = threadIdx.x; b < np; b += blockDim.x) h[b] = 0;
        __syncthreads();
    }
    for (i64 j = blockIdx.x * (i64)blockDim.x + threadIdx.x; j < mx; j += (i64)gridDim.x * blockDim.x) {
        i64 x = row_of_t(xrow, nx, j);
        i32 p = part[x];
        i32 y = xadj[j];
        i64 a = yrow[y], b = yrow[y + 1];
        i64 lo = a, hi = b;
        while (lo < hi) {  // first entry with part >= p
            i64 c = (lo + hi) >> 1;
            if (part[yps[c]] < p) lo = c + 1; else hi = c;
        }
        i64 s = lo;
        hi = b;
        while (lo < hi) {  // first entry with part > p
            i64 c = (lo + hi) >> 1;
            if (part[yps[c]] <= p) lo = c + 1; else hi = c;
        }
        flo[j] = s;
        flen[j] = (i32)(lo - s);
        if (priv) atomicAdd(&h[p], (unsigned long long)(lo - s - 1));
        else atomicAdd((unsigned long long *)&work[p], (unsigned long long)(lo - s - 1));
    }
    if (priv) {
        __syncthreads();
        for (int b = threadIdx.x; b < np; b += blockDim.x)
            if (h[b]) atomicAdd((unsigned long long *)&work[b], h[b]);
    }
}

__global__ void k_lpt_keys(const u64 *work, i32 np, u64 maxw, u64 *keys, i32 *vals, u64 *wmax, u64 *wsum) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < np; p += (i64)gridDim.x * blockDim.x) {
        keys[p] = maxw - work[p];
        vals[p] = (i32)p;
        atomicMax((unsigned long long *)wmax, (unsigned long long)work[p]);
        atomicAdd((unsigned long long *)wsum, (unsigned long long)work[p]);
    }
}

__global__ void k_max_u64(const u64 *a, i64 n, u64 *out) {
    u64 m = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) m = a[i] > m ? a[i] : m;
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        u64 o = __shfl_down(m, d, WAVE);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long *)out, (unsigned long long)m);
}

// ------------------------------------------------------------------ host

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Default P and the work-efficiency clamp of Section 4.2 (tip: P at most the
// wedge total over n log2 n, n = vertices of the peeled side).
static int tip_partitions(const pbng_opts &o, u64 wedge_total, i64 nx) {
    if (o.P > 0) return o.P;
    int P = 150;
    double nlogn = (double)nx * std::log2((double)std::max<i64>(nx, 2));
    double cap = nlogn > 0 ? std::floor((double)wedge_total / nlogn) : 1.0;
    if (cap < 1) cap = 1;
    if (P > cap) P = (int)cap;
    return std::max(P, 1);
}

void tip_decompose(Ctx &c, const DevGraph &G, int side, const pbng_opts &o, u64 *theta) {
    hipStream_t s = c.stream;
    const i64 nx = side == 0 ? G.n_u : G.n_v;
    const i64 ny = side == 0 ? G.n_v : G.n_u;
    const i64 m = G.m;
    const i64 xoff = side == 0 ? 0 : G.n_u;
    if (nx == 0) return;
    const i64 *xrow = side == 0 ? G.urow : G.vrow;
    const i32 *xadj = side == 0 ? G.ucol : G.vadj;
    const i64 *yrow = side == 0 ? G.vrow : G.urow;
    const i32 *yadj0 = side == 0 ? G.vadj : G.ucol;
    const bool dynamic = !(o.flags & PBNG_F_NO_DYNAMIC);
    const bool batch = !(o.flags & PBNG_F_NO_BATCH);
    double t0 = now_ms();

    // ---- counting
    u64 *sup = c.alloc<u64>(nx);
    c.stats.wedges_count += count_side(c, G, side, o, sup);
    PBNG_HIP(hipStreamSynchronize(s));
    double t1 = now_ms();
    c.stats.ms_count = t1 - t0;

    // ---- state
    unsigned char *st = c.alloc<unsigned char>(nx);
    i32 *part = c.alloc<i32>(nx);
    u64 *init = c.alloc<u64>(nx);
    u64 *w = c.alloc<u64>(nx);
    u64 *wsnap = c.alloc<u64>(nx);
    i32 *ydeg = c.alloc<i32>(ny);
    i32 *ylen = c.alloc<i32>(ny);
    unsigned char *ydirty = c.alloc<unsigned char>(ny + 4);
    i32 *dirty = c.alloc<i32>(ny);
    i32 *yadj = c.alloc<i32>(m);
    i32 *F = c.alloc<i32>(nx);
    i32 *F2 = c.alloc<i32>(nx);
    i32 *bins = c.alloc<i32>(5 * nx);
    u64 *wi = c.alloc<u64>(nx);
    TipCtl *ctl = c.alloc<TipCtl>(1);
    PBNG_HIP(hipMemsetAsync(st, 0, nx, s));
    PBNG_HIP(hipMemsetAsync(ydirty, 0, ny + 4, s));
    PBNG_HIP(hipMemsetAsync(ctl, 0, sizeof(TipCtl), s));
    if (m) PBNG_HIP(hipMemcpyAsync(yadj, yadj0, sizeof(i32) * m, hipMemcpyDeviceToDevice, s));
    if (ny) hipLaunchKernelGGL(k_degrees_y, dim3(grid_1d(ny)), dim3(256), 0, s, yrow, ny, ydeg, ylen);
    hipLaunchKernelGGL(k_work_full, dim3(grid_1d(nx * WAVE)), dim3(256), 0, s, xrow, xadj, (const i32 *)ydeg,
                       (const unsigned char *)nullptr, nx, w);
    PBNG_LAUNCH_CHECK();
    u64 *tmp = c.alloc<u64>(2);
    PBNG_HIP(hipMemsetAsync(tmp, 0, 2 * sizeof(u64), s));
    hipLaunchKernelGGL(k_min_deg_sum, dim3(grid_1d(nx)), dim3(256), 0, s, xrow, xadj, (const i32 *)ydeg, nx, tmp);
    PBNG_LAUNCH_CHECK();
    // Section 5.1: a round recounts when its active set's wedges exceed the
    // counting bound (a positive recount_w replaces the bound; negative: never)
    const u64 wedge_cnt_bound = o.recount_w == 0 ? read_scalar<u64>(c, tmp)
                                                 : (o.recount_w < 0 ? ~0ull : (u64)o.recount_w);
    const u64 wedge_total = reduce_sum_u64(c, w, nx);
    const int P = tip_partitions(o, wedge_total, nx);
    c.stats.P_used = P;
    {
        double one = 1.0;
        PBNG_HIP(hipMemcpyAsync(&ctl->scale, &one, sizeof(double), hipMemcpyHostToDevice, s));
    }
    // dense scratch for heavy active vertices
    // key-range path: H_WG_PER_CU workgroups per CU, H_OVF shared sets of
    // overflow counters, the id span of each of its vertices
    const int slots = H_WG_PER_CU * c.num_cu;
    u32 *dcnt = c.alloc<u32>((i64)H_OVF * nx);
    i32 *dtouch = c.alloc<i32>((i64)H_OVF * nx);
    u32 *dlock = c.alloc<u32>(H_OVF);
    i32 *kspan = c.alloc<i32>(2 * nx);
    PBNG_HIP(hipMemsetAsync(dcnt, 0, sizeof(u32) * H_OVF * nx, s));
    PBNG_HIP(hipMemsetAsync(dlock, 0, sizeof(u32) * H_OVF, s));
    unsigned char *alive_label = c.alloc<unsigned char>(G.n);
    u64 *sup_label = c.alloc<u64>(G.n);
    u64 *rmin = c.alloc<u64>(2);
    // learned rule: predicted tip numbers from the initial graph
    u64 *that = nullptr;
    double *one_dev = nullptr;
    c.stats.bound_rule_used = (o.bound_rule == PBNG_BOUND_RANDOM || o.bound_rule == PBNG_BOUND_PAPER) ? o.bound_rule
                                                                                                 : PBNG_BOUND_PLAIN;
    if (o.bound_rule == PBNG_BOUND_LEARNED && (c.mlp_ready || c.tip_hint)) {
        that = c.alloc<u64>(nx);
        if (c.tip_hint)  // predictions supplied by the caller
            PBNG_HIP(hipMemcpyAsync(that, c.tip_hint, sizeof(u64) * nx, hipMemcpyDeviceToDevice, s));
        else
            learned_theta_hat(c, G, side, sup, that);
        one_dev = c.alloc<double>(1);
        const double one = 1.0;
        PBNG_HIP(hipMemcpyAsync(one_dev, &one, sizeof(double), hipMemcpyHostToDevice, s));
        c.stats.bound_rule_used = PBNG_BOUND_LEARNED;
    }
    // LDS key tiles for heavy active vertices (one 512-lane workgroup per
    // CU): 2^16 keys with packed 16-bit counters while every degree is below
    // 2^16 (a count c(x, x') never exceeds the degree of x), else 2^15 keys
    // with 32-bit counters
    const bool pack16 = G.maxdeg < 65536;
    const int tile_log = pack16 ? TILE_LOG : TILE_LOG - 1;
    const i32 ntiles = (i32)((nx + (i64(1) << tile_log) - 1) >> tile_log);
    const int tslots = c.num_cu;
    // active vertices above huge_w wedges take the key tiles; default: at
    // least 16384 wedges per key tile on average
    const u64 huge_w = o.tile_w == 0 ? std::max<u64>((u64)HUGE_W, (u64)ntiles * 16384u)
                                     : (o.tile_w < 0 ? ~0ull : (u64)o.tile_w);
    u32 *hoff = c.alloc<u32>(nx + 1);
    u32 *htotal = c.alloc<u32>(1);

    PeelArgs pa{};
    pa.xrow = xrow;
    pa.xadj = xadj;
    pa.yrow = yrow;
    pa.yadj = yadj;
    pa.ylen = ylen;
    pa.nitems = ctl->nbin;
    pa.next = ctl->next;
    pa.st = st;
    pa.sup = sup;
    pa.wi = wi;
    pa.bound = &ctl->bound;
    pa.nnf = &ctl->nF2;
    pa.dcnt = dcnt;
    pa.dtouch = dtouch;
    pa.dlock = dlock;
    pa.kspan = kspan;
    pa.hprobe = (o.flags & PBNG_F_SHORT_PROBE) ? 1 : H_PROBE;
    pa.ntiles = ntiles;
    pa.nx = nx;
    pa.tnext = &ctl->tnext;
    pa.wedges = &ctl->wedges;
    pa.kc = c.kctr + PBNG_K_TIP_PEEL;

    struct HostView {
        u32 nF;
        u64 wF;
    };
    i64 n_alive = nx;
    int pid = 0;
    u64 rho = 0, recounts = 0, recount_wedges = 0;
    const bool trace = getenv("PBNG_TRACE") != nullptr;
    u64 trace_w = 0;
    double trace_t = now_ms();
    const int gx = grid_1d(nx);
    auto item_work = [&](i32 *cur) {
        hipLaunchKernelGGL(k_item_work, dim3(grid_1d((i64)nx * WAVE)), dim3(256), 0, s, (const i32 *)cur,
                           (const u32 *)&ctl->nF, xrow, xadj, (const i64 *)yrow, (const i32 *)yadj, (const i32 *)ylen, wi,
                           &ctl->wF, bins, nx, ctl->nbin, huge_w, kspan);
        PBNG_LAUNCH_CHECK();
    };
    // Levels of single-value partitions (~0 for ordinary ranges).  When what
    // is left is a small, heavy dense core (at most LEVEL_MAX_ALIVE vertices,
    // LEVEL_MIN_WORK wedges of work or more, LEVEL_MIN_AVG or more per
    // vertex), its fine-grained peeling would run on one workgroup; instead
    // the coarse-grained loop goes on one support level per partition, each
    // peeled by the whole GPU, and those partitions skip the fine-grained
    // phase (the partition count may then exceed P).
    u64 *plev = c.alloc<u64>((i64)P + nx + 1);
    fill<u64>(c, plev, ~0ull, (i64)P + nx + 1);
    // exclusive upper bound theta(i+1) of every partition (schedule output)
    u64 *pbound = c.sched_part ? c.alloc<u64>((i64)P + nx + 1) : nullptr;
    u64 *alive_work = c.alloc<u64>(1);
    bool level_mode = false;
    // opts.level_alive: 0 = the defaults above; positive = single levels as
    // soon as at most that many vertices are alive, whatever their work;
    // negative = never.  The paper's rule (PBNG_BOUND_PAPER) has no levels.
    const bool paper_rule = o.bound_rule == PBNG_BOUND_PAPER;
    const i64 level_max_alive =
        paper_rule || o.level_alive < 0 ? -1 : (o.level_alive > 0 ? (i64)o.level_alive : LEVEL_MAX_ALIVE);
    const u64 level_min_work = o.level_alive > 0 ? 0 : LEVEL_MIN_WORK;
    const u64 level_min_avg = o.level_alive > 0 ? 0 : LEVEL_MIN_AVG;
    // ---- coarse-grained rounds
    // A push round peels the current active set Fa by wedge traversal and
    // sweeps the next one into Fb; gridF bounds the grids (the active set's
    // size on the host-driven path, every vertex when captured).
    auto push_round = [&](hipStream_t rs, i32 *Fa, i32 *Fb, i64 gridF) {
        (void)Fa;
        pa.items = bins;
        pa.nf = Fb;
        PeelArgs pd = pa;
        pd.items = bins + 3 * nx;
        PeelArgs pt = pa;
        pt.items = bins + 2 * nx;
        PeelArgs pm = pa;
        pm.items = bins + nx;
        {
            PeelArgs pk = pd;
            pk.kc = c.kctr + PBNG_K_TIP_TILED;
            c.kbegin(PBNG_K_TIP_TILED, rs);
            const dim3 tg((unsigned)std::min<i64>(tslots, gridF * ntiles));
            if (pack16)
                hipLaunchKernelGGL((k_tip_peel_tiled<TILE_LOG, true>), tg, dim3(512), 0, rs, pk, 3);
            else
                hipLaunchKernelGGL((k_tip_peel_tiled<TILE_LOG - 1, false>), tg, dim3(512), 0, rs, pk, 3);
            c.kend(PBNG_K_TIP_TILED, rs);
        }
        c.kbegin(PBNG_K_TIP_PEEL, rs);
        hipLaunchKernelGGL(k_range_split, dim3(1), dim3(1024), 0, rs, (const i32 *)pt.items, (const u32 *)ctl->nbin, 2,
                           (const u64 *)wi, hoff, htotal);
        c.kend(PBNG_K_TIP_PEEL, rs);
        {
            PeelArgs ph = pt;
            ph.kc = c.kctr + PBNG_K_TIP_HRANGE;
            c.kbegin(PBNG_K_TIP_HRANGE, rs);
            hipLaunchKernelGGL((k_tip_peel_hrange<H_LOGCAP, H_BLOCK>), dim3(std::min<i64>(slots, gridF * H_RANGE_MAX)),
                               dim3(H_BLOCK), 0, rs,
                               ph, 2, (const u32 *)hoff, (const u32 *)htotal);
            c.kend(PBNG_K_TIP_HRANGE, rs);
        }
        c.kbegin(PBNG_K_TIP_PEEL, rs);
        {
            PeelArgs pp = pa;
            pp.items = bins + 4 * nx;
            hipLaunchKernelGGL(k_tip_peel_pairs, dim3(std::min<i64>((i64)c.num_cu * 8, (gridF + 3) / 4)), dim3(256), 0, rs, pp,
                               4);
        }
        hipLaunchKernelGGL((k_tip_peel_hash<256, 13>), dim3(std::min<i64>((i64)c.num_cu * 2, gridF)), dim3(256), 0, rs, pm, 1);
        hipLaunchKernelGGL((k_tip_peel_hash<64, 10>), dim3(std::min<i64>((i64)c.num_cu * 16, gridF)), dim3(64), 0, rs, pa, 0);
        c.kend(PBNG_K_TIP_PEEL, rs);
        PBNG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sweep_frontier, dim3(gx), dim3(256), 0, rs, (const unsigned char *)st, (const u64 *)sup,
                           (const TipCtl *)ctl, nx, Fb, &ctl->nF2);
        PBNG_LAUNCH_CHECK();
    };
    // after the updates: retire Fa, activate Fb, compact the dirty lists,
    // make Fb current and bin it
    // (grid-stride kernels; captured rounds launch at most gcap blocks)
    auto end_round = [&](hipStream_t rs, i32 *Fa, i32 *Fb, i64 gridF, int gcap) {
        hipLaunchKernelGGL(k_retire, dim3(grid_1d(gridF * WAVE, 256, gcap)), dim3(256), 0, rs, (const i32 *)Fa,
                           (const u32 *)&ctl->nF, xrow, xadj, st, ydeg, ydirty, dirty, &ctl->ndirty, dynamic ? 1 : 0);
        hipLaunchKernelGGL(k_activate, dim3(grid_1d(nx, 256, gcap)), dim3(256), 0, rs, (const i32 *)Fb, (const u32 *)&ctl->nF2,
                           st, part, (const TipCtl *)ctl);
        PBNG_LAUNCH_CHECK();
        if (dynamic) {
            hipLaunchKernelGGL(k_compact, dim3(grid_1d((i64)ny * WAVE, 256, gcap)), dim3(256), 0, rs, (const i32 *)dirty,
                               (const u32 *)&ctl->ndirty, yrow, yadj, ylen, ydirty, (const unsigned char *)st);
            PBNG_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_next_round, dim3(1), dim3(1), 0, rs, ctl);
        hipLaunchKernelGGL(k_item_work, dim3(grid_1d((i64)nx * WAVE, 256, gcap)), dim3(256), 0, rs, (const i32 *)Fb,
                           (const u32 *)&ctl->nF, xrow, xadj, (const i64 *)yrow, (const i32 *)yadj, (const i32 *)ylen, wi,
                           &ctl->wF, bins, nx, ctl->nbin, huge_w, kspan);
        PBNG_LAUNCH_CHECK();
    };
    // Section 5.1: supports of the remaining graph by counting (the active
    // set is already retired), then the active set below the bound
    auto recount_remaining = [&]() {
        hipLaunchKernelGGL(k_alive_label, dim3(grid_1d(G.n)), dim3(256), 0, s, (const unsigned char *)st, (const i32 *)G.gid,
                           G.n, xoff, nx, alive_label);
        PBNG_LAUNCH_CHECK();
        recount_wedges += count_pass(c, G, sup_label, nullptr, alive_label);
        hipLaunchKernelGGL(k_from_label, dim3(gx), dim3(256), 0, s, (const u64 *)sup_label, (const i32 *)G.label, xoff, nx,
                           (const unsigned char *)st, sup);
        PBNG_LAUNCH_CHECK();
        ++recounts;
        hipLaunchKernelGGL(k_frontier, dim3(gx), dim3(256), 0, s, st, (const u64 *)sup, (const u64 *)w, init, wsnap, part, nx,
                           ctl, pid, 0, F);
        PBNG_LAUNCH_CHECK();
        item_work(F);
    };
    // captured rounds; host-driven with PBNG_F_HOST_ROUNDS, while tracing,
    // and under kernel-class timing (events recorded inside a graph cannot
    // be timed here: kernels are the same either way)
    const bool host_rounds = (o.flags & (PBNG_F_HOST_ROUNDS | PBNG_F_KERNEL_TIMING)) != 0 || trace;
    GraphExec rounds_exec;
    {
        const u64 init_ctl[2] = {(u64)nx, wedge_cnt_bound};  // alive, wbound
        PBNG_HIP(hipMemcpyAsync(&ctl->alive, init_ctl, sizeof(init_ctl), hipMemcpyHostToDevice, s));
    }
    if (!host_rounds) {
        hipStream_t cs = c.capture_stream();
        PBNG_HIP(hipStreamSynchronize(s));
        PBNG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        i32 *Fa = F, *Fb = F2;
        for (int r = 0; r < TIP_GRAPH_K; ++r) {
            hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, cs, ctl, batch ? 1 : 0);
            push_round(cs, Fa, Fb, c.num_cu * 4);
            end_round(cs, Fa, Fb, nx, c.num_cu * 8);
            std::swap(Fa, Fb);
        }
        const hipError_t le = hipGetLastError();
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        PBNG_HIP(le);
        PBNG_HIP(ee);
        const hipError_t ie = hipGraphInstantiate(&rounds_exec.e, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        PBNG_HIP(ie);
    }
    while (n_alive > 0) {
        const bool at_last = (P - pid) <= 1;
        // work estimate of every alive vertex with the current live degrees
        // (not needed once partitions are single levels)
        if (!level_mode) {
            hipLaunchKernelGGL(k_work_full, dim3(grid_1d(nx * WAVE)), dim3(256), 0, s, xrow, xadj, (const i32 *)ydeg,
                               (const unsigned char *)st, nx, w);
            PBNG_LAUNCH_CHECK();
        }
        if (!level_mode && n_alive <= level_max_alive) {
            PBNG_HIP(hipMemsetAsync(alive_work, 0, sizeof(u64), s));
            hipLaunchKernelGGL(k_alive_work, dim3(std::min<i64>(grid_1d(nx), 512)), dim3(256), 0, s,
                               (const unsigned char *)st, (const u64 *)w, nx, alive_work);
            PBNG_LAUNCH_CHECK();
            const u64 wr = read_scalar<u64>(c, alive_work);
            level_mode = wr >= level_min_work && wr / (u64)n_alive >= level_min_avg;
            if (trace)
                fprintf(stderr, "[pbng-trace] partition %d: %lld alive, work %llu -> %s\n", pid, (long long)n_alive,
                        (unsigned long long)wr, level_mode ? "single levels" : "ranges");
        }
        const bool last = at_last && !level_mode;
        if (level_mode) {
            u64 init2[2] = {~0ull, 0};
            PBNG_HIP(hipMemcpyAsync(rmin, init2, sizeof(init2), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_random_bound, dim3(std::min(gx, 512)), dim3(256), 0, s, (const u64 *)sup, (const unsigned char *)st, nx,
                               rmin, rmin + 1);
            hipLaunchKernelGGL(k_level_bound, dim3(1), dim3(1), 0, s, ctl, (const u64 *)rmin, plev + pid);
            PBNG_LAUNCH_CHECK();
        } else if (!last) {
            if (o.bound_rule == PBNG_BOUND_RANDOM) {
                u64 init2[2] = {~0ull, 0};
                PBNG_HIP(hipMemcpyAsync(rmin, init2, sizeof(init2), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_random_bound, dim3(std::min(gx, 512)), dim3(256), 0, s, (const u64 *)sup, (const unsigned char *)st, nx,
                                   rmin, rmin + 1);
                hipLaunchKernelGGL(k_random_pick, dim3(1), dim3(1), 0, s, ctl, (const u64 *)rmin, (const u64 *)(rmin + 1),
                                   (u64)o.seed, pid);
                PBNG_LAUNCH_CHECK();
            } else if (that) {
                // work-weighted quantile of the predicted tip numbers, kept
                // above the smallest alive support so the partition is never empty
                weighted_select(c, that, w, st, ST_ALIVE, nx, nullptr, one_dev, P - pid, &ctl->s, &ctl->est_init);
                u64 init2[2] = {~0ull, 0};
                PBNG_HIP(hipMemcpyAsync(rmin, init2, sizeof(init2), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_random_bound, dim3(std::min(gx, 512)), dim3(256), 0, s, (const u64 *)sup, (const unsigned char *)st, nx,
                                   rmin, rmin + 1);
                hipLaunchKernelGGL(k_learned_guard, dim3(1), dim3(1), 0, s, ctl, (const u64 *)rmin);
                PBNG_LAUNCH_CHECK();
            } else {
                // ranges also end at a vertex-count target: a partition of many
                // light vertices peels one level at a time in the
                // fine-grained phase, with a pass over its vertices per level,
                // so its cost grows with (vertices x levels), which the work
                // estimate does not see; the target keeps such partitions
                // near the size whose state fits in LDS
                const u64 cnt_target = paper_rule ? 0
                    : std::max<u64>((u64)FD_LDS_NI, (u64)(2 * n_alive / std::max<i64>(P - pid, 1)));
                weighted_select(c, sup, w, st, ST_ALIVE, nx, nullptr, &ctl->scale, P - pid, &ctl->s, &ctl->est_init,
                                cnt_target);
            }
        }
        hipLaunchKernelGGL(k_set_bound, dim3(1), dim3(1), 0, s, ctl, last ? 1 : 0, (i32)pid);
        if (pbound) hipLaunchKernelGGL(k_record_bound, dim3(1), dim3(1), 0, s, (const TipCtl *)ctl, pbound + pid);
        hipLaunchKernelGGL(k_frontier, dim3(gx), dim3(256), 0, s, st, (const u64 *)sup, (const u64 *)w, init, wsnap, part,
                           nx, ctl, pid, 1, F);
        PBNG_LAUNCH_CHECK();
        item_work(F);
        if (!host_rounds) {
            // replays until the partition's active set is empty; a replay
            // that handed a set to a recount is followed by the recount here
            for (;;) {
                PBNG_HIP(hipGraphLaunch(rounds_exec.e, s));
                TipCtl h;
                PBNG_HIP(hipMemcpyAsync(&h, ctl, sizeof(TipCtl), hipMemcpyDeviceToHost, s));
                PBNG_HIP(hipStreamSynchronize(s));
                n_alive = (i64)h.alive;
                if (h.recount) {
                    recount_remaining();
                    const u32 zero = 0;
                    PBNG_HIP(hipMemcpyAsync(&ctl->recount, &zero, sizeof(u32), hipMemcpyHostToDevice, s));
                    continue;
                }
                if (h.nF == 0) break;
            }
        } else {
            HostView hv;
            PBNG_HIP(hipMemcpyAsync(&hv.nF, &ctl->nF, sizeof(u32), hipMemcpyDeviceToHost, s));
            PBNG_HIP(hipMemcpyAsync(&hv.wF, &ctl->wF, sizeof(u64), hipMemcpyDeviceToHost, s));
            PBNG_HIP(hipStreamSynchronize(s));
            while (hv.nF > 0) {
                ++rho;
                const u32 nF = hv.nF;
                const int gw = grid_1d((i64)nF * WAVE);
                if ((i64)nF == n_alive) {
                    // everything left joins this partition: no updates needed
                    hipLaunchKernelGGL(k_retire, dim3(gw), dim3(256), 0, s, (const i32 *)F, (const u32 *)&ctl->nF, xrow, xadj,
                                       st, ydeg, ydirty, dirty, &ctl->ndirty, 0);
                    PBNG_LAUNCH_CHECK();
                    n_alive = 0;
                    hipLaunchKernelGGL(k_next_round, dim3(1), dim3(1), 0, s, ctl);
                    break;
                }
                if (batch && hv.wF > wedge_cnt_bound) {
                    // Section 5.1: recount the remaining graph instead of peeling
                    hipLaunchKernelGGL(k_retire, dim3(gw), dim3(256), 0, s, (const i32 *)F, (const u32 *)&ctl->nF, xrow, xadj,
                                       st, ydeg, ydirty, dirty, &ctl->ndirty, dynamic ? 1 : 0);
                    PBNG_LAUNCH_CHECK();
                    n_alive -= nF;
                    if (dynamic) {
                        hipLaunchKernelGGL(k_compact, dim3(grid_1d((i64)ny * WAVE)), dim3(256), 0, s, (const i32 *)dirty,
                                           (const u32 *)&ctl->ndirty, yrow, yadj, ylen, ydirty, (const unsigned char *)st);
                        PBNG_LAUNCH_CHECK();
                    }
                    hipLaunchKernelGGL(k_next_round, dim3(1), dim3(1), 0, s, ctl);
                    recount_remaining();
                } else {
                    push_round(s, F, F2, nF);
                    if (trace) {
                        u32 nb[4];
                        u64 wtot;
                        PBNG_HIP(hipMemcpyAsync(nb, ctl->nbin, sizeof(nb), hipMemcpyDeviceToHost, s));
                        PBNG_HIP(hipMemcpyAsync(&wtot, &ctl->wedges, sizeof(u64), hipMemcpyDeviceToHost, s));
                        PBNG_HIP(hipStreamSynchronize(s));
                        double tnow = now_ms();
                        fprintf(stderr,
                                "[pbng-trace] part %d round %llu nF %u wF %llu bins %u/%u/%u/%u wedges %llu ms %.3f\n", pid,
                                (unsigned long long)rho, nF, (unsigned long long)hv.wF, nb[0], nb[1], nb[2], nb[3],
                                (unsigned long long)(wtot - trace_w), tnow - trace_t);
                        trace_w = wtot;
                        trace_t = tnow;
                    }
                    end_round(s, F, F2, nF, 16384);
                    n_alive -= nF;
                    std::swap(F, F2);
                }
                PBNG_HIP(hipMemcpyAsync(&hv.nF, &ctl->nF, sizeof(u32), hipMemcpyDeviceToHost, s));
                PBNG_HIP(hipMemcpyAsync(&hv.wF, &ctl->wF, sizeof(u64), hipMemcpyDeviceToHost, s));
                PBNG_HIP(hipStreamSynchronize(s));
            }
        }
        hipLaunchKernelGGL(k_part_work, dim3(std::min<i64>(grid_1d(nx), 512)), dim3(256), 0, s, (const unsigned char *)st,
                           (const i32 *)part, (const u64 *)wsnap, nx, pid, ctl);
        hipLaunchKernelGGL(k_scale, dim3(1), dim3(1), 0, s, ctl);
        PBNG_LAUNCH_CHECK();
        ++pid;
    }
    const i32 np = pid;
    c.stats.wedges_cd = read_scalar<u64>(c, &ctl->wedges) + recount_wedges;
    if (!host_rounds) rho += read_scalar<u64>(c, &ctl->rounds);
    c.stats.rho = rho;
    c.stats.recounts = recounts;
    c.stats.partitions = np;
    if (c.sched_part) {
        PBNG_HIP(hipMemcpyAsync(c.sched_part, part, sizeof(i32) * nx, hipMemcpyDeviceToDevice, s));
        PBNG_HIP(hipMemcpyAsync(c.sched_init, init, sizeof(u64) * nx, hipMemcpyDeviceToDevice, s));
        const i32 nb = std::min<i32>(np, c.sched_cap);
        if (nb > 0) PBNG_HIP(hipMemcpyAsync(c.sched_bounds, pbound, sizeof(u64) * nb, hipMemcpyDeviceToDevice, s));
        c.sched_np = np;
    }
    double t2 = now_ms();
    c.stats.ms_cd = t2 - t1;

    // ---- FD preparation: vertices and Y lists grouped by partition
    u64 *pk = c.alloc<u64>(std::max<i64>(nx, m));
    i32 *pv = c.alloc<i32>(std::max<i64>(nx, m));
    u32 *pcount = c.alloc<u32>(np);
    PBNG_HIP(hipMemsetAsync(pcount, 0, sizeof(u32) * np, s));
    hipLaunchKernelGGL(k_part_keys, dim3(gx), dim3(256), 0, s, (const i32 *)part, nx, pk, pv);
    hist_add_u32(c, part, nx, np, pcount);
    PBNG_LAUNCH_CHECK();
    u64 *sk;
    i32 *xs;
    radix_sort_u64(c, pk, pv, nx, bits_for((u64)np), &sk, &xs);
    i64 *pc64 = c.alloc<i64>(np);
    i64 *poff = c.alloc<i64>(np + 1);
    hipLaunchKernelGGL(k_u32_to_i64_t, dim3(grid_1d(np)), dim3(256), 0, s, (const u32 *)pcount, (i64)np, pc64);
    exclusive_scan<i64>(c, pc64, poff, np);
    i32 *loc = c.alloc<i32>(nx);
    hipLaunchKernelGGL(k_loc, dim3(gx), dim3(256), 0, s, (const i32 *)xs, (const i32 *)part, (const i64 *)poff, nx, loc);
    PBNG_LAUNCH_CHECK();
    u64 *yk = c.alloc<u64>(m);
    i32 *yv = c.alloc<i32>(m);
    i32 *yps = yv;
    i64 *flo = c.alloc<i64>(m);
    i32 *flen = c.alloc<i32>(m);
    u64 *work = c.alloc<u64>(np);
    PBNG_HIP(hipMemsetAsync(work, 0, sizeof(u64) * np, s));
    if (m) {
        hipLaunchKernelGGL(k_ypart_keys, dim3(grid_1d(m)), dim3(256), 0, s, yrow, yadj0, (const i32 *)part, ny, m, np, yk, yv);
        PBNG_LAUNCH_CHECK();
        u64 *ysk;
        radix_sort_u64(c, yk, yv, m, bits_for((u64)ny * (u64)np), &ysk, &yps);
        hipLaunchKernelGGL(k_fd_segments, dim3(std::min<i64>(grid_1d(m), (i64)c.num_cu * 8)), dim3(256), 0, s, xrow, xadj,
                           nx, m, yrow, (const i32 *)yps, (const i32 *)part, flo, flen, work, np);
        PBNG_LAUNCH_CHECK();
    }
    // LPT order
    u64 *wm = c.alloc<u64>(3);
    PBNG_HIP(hipMemsetAsync(wm, 0, 3 * sizeof(u64), s));
    hipLaunchKernelGGL(k_max_u64, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)work, (i64)np, wm);
    const u64 maxw = read_scalar<u64>(c, wm);
    u64 *lk = c.alloc<u64>(np);
    i32 *lv = c.alloc<i32>(np);
    hipLaunchKernelGGL(k_lpt_keys, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)work, np, maxw, lk, lv, wm + 1, wm + 2);
    PBNG_LAUNCH_CHECK();
    u64 *lks;
    i32 *queue;
    radix_sort_u64(c, lk, lv, np, bits_for(maxw), &lks, &queue);
    c.stats.fd_work_max = read_scalar<u64>(c, wm + 1);
    c.stats.fd_work_sum = read_scalar<u64>(c, wm + 2);
    // largest partition for scratch sizing
    i64 *maxni_d = reinterpret_cast<i64 *>(c.alloc<u64>(1));
    PBNG_HIP(hipMemsetAsync(maxni_d, 0, sizeof(u64), s));
    hipLaunchKernelGGL(k_max_u64, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)pc64, (i64)np, (u64 *)maxni_d);
    const i64 maxni = std::max<i64>(read_scalar<i64>(c, maxni_d), 1);
    PBNG_HIP(hipStreamSynchronize(s));
    double t3 = now_ms();
    c.stats.ms_fd_prep = t3 - t2;

    // ---- FD
    const int fdblocks = (int)std::min<i64>(np, (i64)c.num_cu * 2);
    FdArgs fa{};
    fa.xrow = xrow;
    fa.xadj = xadj;
    fa.xs = xs;
    fa.poff = poff;
    fa.loc = loc;
    fa.yps = yps;
    fa.flo = flo;
    fa.flen = flen;
    fa.queue = queue;
    fa.np = np;
    fa.head = c.alloc<u32>(1);
    PBNG_HIP(hipMemsetAsync(fa.head, 0, sizeof(u32), s));
    fa.init = init;
    fa.plev = plev;
    fa.theta = theta;
    fa.maxni = maxni;
    fa.pack16 = pack16 ? 1 : 0;
    fa.lsup = c.alloc<u64>((i64)fdblocks * maxni);
    fa.lst = c.alloc<unsigned char>((i64)fdblocks * maxni);
    fa.lcnt = c.alloc<u32>((i64)fdblocks * maxni);
    fa.ltouch = c.alloc<i32>((i64)fdblocks * maxni);
    fa.lbatch = c.alloc<i32>((i64)fdblocks * maxni);
    fa.lheavy = c.alloc<i32>((i64)fdblocks * maxni);
    fa.wedges = c.alloc<u64>(1);
    fa.kc = c.kctr + PBNG_K_FD;
    PBNG_HIP(hipMemsetAsync(fa.wedges, 0, sizeof(u64), s));
    c.kbegin(PBNG_K_FD);
    hipLaunchKernelGGL(k_tip_fd, dim3(fdblocks), dim3(FD_BLOCK), 0, s, fa);
    c.kend(PBNG_K_FD);
    PBNG_LAUNCH_CHECK();
    c.stats.wedges_fd = read_scalar<u64>(c, fa.wedges);
    c.stats.ms_fd = now_ms() - t3;
    c.stats.wedges = c.stats.wedges_count + c.stats.wedges_cd + c.stats.wedges_fd;
}

}  // namespace pbng
