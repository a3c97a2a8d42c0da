// Butterfly counting by priority wedge traversal (Algorithm 1) and BE-Index
// construction inside the same traversal (Section 2.3, "Construction").
//
// For a start vertex s (a label), every wedge s -> mid -> last with
// last < min(s, mid) is walked; the lasts of one mid form the prefix of the
// sorted N_mid whose length prep stored in lpl.  wc[last] counts the wedges
// per (s, last).  A (s, last) pair with wc >= 2 is one maximal priority bloom
// with bloom number wc; its C(wc, 2) butterflies contain s and last once each
// and every mid wc - 1 times; the edges (s, mid) and (mid, last) of each of
// its wedges are twins and each lies in wc - 1 of its butterflies.
//
// Work mapping: starts are binned by their wedge count W_s.
//   small  (W_s <= 512)  : one 64-lane workgroup per start, LDS hash
//   medium (W_s <= 4096) : one 256-lane workgroup per start, LDS hash
//   large                : persistent 256-lane workgroups, each with a dense
//                          counter array over all labels in HBM plus a list of
//                          the labels it touched
// Inside a start, the (mid, prefix) segments are processed BLOCK at a time:
// a block scan of the prefix lengths lets each lane take a run of
// consecutive wedges, found by one binary search over the segment starts and
// a forward walk, whatever the degree mix.
#include "pbng_internal.h"

#include <algorithm>

#include "dev_common.h"

namespace pbng {

enum : int {
    M_VERTEX = 1,   // per-vertex supports (by label)
    M_EDGE = 2,     // per-edge supports (by edge id)
    M_BE_SIZE = 4,  // count blooms / pairs per start
    M_BE_FILL = 8,  // emit blooms and twin pairs (and per-edge supports)
    M_XSIDE = 16,   // per-vertex supports of one side X only, without the
                    // butterflies whose two X vertices are both hubs
};

// Vertex classes for M_XSIDE (by label)
enum : unsigned char { LC_Y = 0, LC_X = 1, LC_XHUB = 2 };

constexpr u32 NO_BLOOM = 0xFFFFFFFFu;

struct CountArgs {
    const i64 *loff;
    const i32 *ladj, *leid, *lpl;
    const i64 *wsum;             // wedges per start (upper bound when filtered)
    const unsigned char *alive;  // by label; null = all alive
    const unsigned char *lclass; // M_XSIDE: LC_* by label
    u64 *sup_label;              // M_VERTEX
    u64 *sup_edge;               // M_EDGE / M_BE_FILL
    const i32 *starts;           // work list of this bin
    i64 nstarts;
    u32 *next;                   // work counter
    i64 *bcnt, *pcnt;            // M_BE_SIZE: per start
    const i64 *bbase, *pbase;    // M_BE_FILL: exclusive prefix per start
    i64 *boff;                   // M_BE_FILL: first pair of each bloom
    u32 *bk;                     // M_BE_FILL: bloom number
    i32 *bedge;                  // M_BE_FILL: twin pairs (2 edge ids per pair)
    i32 *pbloom;                 // M_BE_FILL: bloom of each pair
    u32 *dcnt;                   // dense accumulators [slots * n]
    i32 *dbid;                   // [slots * n]
    i32 *dtouch;                 // [slots * n]
    u32 *dntouch;                // [slots]
    i64 n;
    u64 *wedges;                 // wedges walked
    KCounters *kc;               // algorithmic-work counters of this class
};


// ------------------------------------------------------------------ traversal

struct ChunkSmem {
    i32 *pre;    // [BLOCK] inclusive prefix of the chunk's prefix lengths
    i64 *moff;   // [BLOCK] first entry of each mid's list
    u64 *agg;    // [BLOCK] per-mid aggregate
    i32 *wave;   // [BLOCK / WAVE]
    u64 *red;    // [BLOCK / WAVE]
    i64 *bcast;  // [1]
};

// Visits the wedges k0 .. k0 + UNR - 1 of a chunk whose segment wedge counts
// have inclusive prefix pre[0..last] and whose runs start at ladj[moff[l]]:
// one binary search finds the segment of k0, the rest of the run walks
// forward (reading the next prefix only where a segment ends), the far ends
// are loaded together (a wedge past tot reads ladj[0], which exists whenever
// tot > 0), then fn(seg, pos, far end) runs for each wedge below tot.
constexpr int CR_UNR = 4;
template <int UNR, class F>
__device__ __forceinline__ void chunk_run(const i32 *ladj, const i32 *pre, const i64 *moff, int last, i32 k0, i32 tot,
                                          F fn) {
    int sq[UNR];
    i64 pq[UNR];
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
        sq[q] = -1;
        pq[q] = 0;
    }
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
                sq[q] = l;
                pq[q] = base + k;
            }
        }
    }
    i32 lq[UNR];
#pragma unroll
    for (int q = 0; q < UNR; ++q) lq[q] = ladj[pq[q]];
#pragma unroll
    for (int q = 0; q < UNR; ++q)
        if (sq[q] >= 0) fn(sq[q], pq[q], lq[q]);
}

// Calls wedge(seg, jmid, last, pos) for every wedge of start s, where jmid is
// the entry of mid in N_s, seg = jmid - chunk base, and pos the entry of last
// in N_mid; chunk_end(cb) runs after each chunk of BLOCK mids, between
// barriers.
template <int BLOCK, class FW, class FC>
__device__ __forceinline__ void for_each_wedge(const CountArgs &a, i32 s, const ChunkSmem &sm, FW wedge, FC chunk_end) {
    const i64 jb = a.loff[s], je = a.loff[s + 1];
    for (i64 cb = jb; cb < je; cb += BLOCK) {
        i64 j = cb + threadIdx.x;
        i32 pl = 0;
        i64 moff = 0;
        if (j < je) {
            i32 mid = a.ladj[j];
            pl = a.lpl[j];
            if (a.alive && !a.alive[mid]) pl = 0;
            moff = a.loff[mid];
        }
        i32 tot;
        i32 incl = block_incl_scan_i32<BLOCK>(pl, sm.wave, tot);
        sm.pre[threadIdx.x] = incl;
        sm.moff[threadIdx.x] = moff;
        __syncthreads();
        for (i32 kb = 0; kb < tot; kb += CR_UNR * BLOCK)
            chunk_run<CR_UNR>(a.ladj, sm.pre, sm.moff, BLOCK - 1, kb + (i32)threadIdx.x * CR_UNR, tot,
                              [&](int seg, i64 pos, i32 last) {
                                  if (a.alive && !a.alive[last]) return;
                                  wedge(seg, cb + seg, last, pos);
                              });
        __syncthreads();
        chunk_end(cb);
        __syncthreads();
    }
}

// One-side counts without hub-hub butterflies.  A butterfly whose highest-
// priority vertex is on side X pairs a start and a last on X; when both are
// hubs the start is a hub (the last has at least its degree), and hub starts
// are never scheduled.  A butterfly whose highest vertex is on Y pairs two X
// mids of a (start, last) on Y; counts are kept packed per last as
// (all mids) + 2^16 (hub mids), and a mid's share excludes the other hub
// mids when it is a hub itself.  Every count is below 2^16 (the host checks
// the maximum degree).
template <int BLOCK, class Acc>
__device__ __forceinline__ void process_start_xside(const CountArgs &a, i32 s, Acc &A, const ChunkSmem &sm, Tally &t) {
    const unsigned char sc = a.lclass[s];
    for_each_wedge<BLOCK>(a, s, sm,
        [&](int, i64 jmid, i32 last, i64) {
            const u32 inc = (sc == LC_Y && a.lclass[a.ladj[jmid]] == LC_XHUB) ? 0x10001u : 1u;
            A.add(last, inc);
            ++t.wedges;
        },
        [&](i64) {});
    if (threadIdx.x == 0) {
        t.segments += (u64)(a.loff[s + 1] - a.loff[s]);
        t.items += 1;
    }
    if (threadIdx.x == 0) sm.bcast[0] = A.entries();
    __syncthreads();
    const i64 ne = sm.bcast[0];
    __syncthreads();
    if (sc != LC_Y) {
        u64 my_start = 0;
        for (i64 i = threadIdx.x; i < ne; i += BLOCK) {
            i32 key;
            u32 v;
            A.entry(i, key, v);
            const u64 cc = v & 0xFFFFu;
            if (key < 0 || cc < 2) continue;
            const u64 b = cc * (cc - 1) / 2;
            my_start += b;
            atomicAdd((unsigned long long *)&a.sup_label[key], (unsigned long long)b);
            ++t.atomics;
        }
        const u64 tt = block_sum_u64<BLOCK>(my_start, sm.red);
        if (threadIdx.x == 0 && tt) {
            atomicAdd((unsigned long long *)&a.sup_label[s], (unsigned long long)tt);
            ++t.atomics;
        }
        __syncthreads();
        return;
    }
    sm.agg[threadIdx.x] = 0;
    __syncthreads();
    for_each_wedge<BLOCK>(a, s, sm,
        [&](int seg, i64 jmid, i32 last, i64) {
            const u32 v = A.cnt(A.find(last));
            const u64 cc = v & 0xFFFFu;
            if (cc < 2) return;
            const u64 hub = v >> 16;
            const u64 share = a.lclass[a.ladj[jmid]] == LC_XHUB ? cc - hub : cc - 1;
            if (share) atomicAdd((unsigned long long *)&sm.agg[seg], (unsigned long long)share);
        },
        [&](i64 cb) {
            const u64 g = sm.agg[threadIdx.x];
            if (g) {
                atomicAdd((unsigned long long *)&a.sup_label[a.ladj[cb + threadIdx.x]], (unsigned long long)g);
                ++t.atomics;
                sm.agg[threadIdx.x] = 0;
            }
        });
}

// Everything done for one start: pass 1 (wedge counts), the per-bloom
// epilogue, pass 2 (mid and edge contributions, twin pairs).
template <int BLOCK, int MODE, class Acc>
__device__ __forceinline__ void process_start(const CountArgs &a, i32 s, Acc &A, const ChunkSmem &sm, Tally &t) {
    if constexpr ((MODE & M_XSIDE) != 0) {
        process_start_xside<BLOCK>(a, s, A, sm, t);
        return;
    }
    for_each_wedge<BLOCK>(a, s, sm, [&](int, i64, i32 last, i64) { A.add(last); ++t.wedges; }, [&](i64) {});
    if (threadIdx.x == 0) {
        t.segments += (u64)(a.loff[s + 1] - a.loff[s]);
        t.items += 1;
    }

    if (threadIdx.x == 0) sm.bcast[0] = A.entries();
    __syncthreads();
    const i64 ne = sm.bcast[0];
    __syncthreads();
    if (MODE & M_BE_FILL) {
        const i64 bb = a.bbase[s], pb = a.pbase[s];
        i64 carry_b = 0, carry_p = 0;
        for (i64 base = 0; base < ne; base += BLOCK) {
            i64 i = base + threadIdx.x;
            i32 key = -1;
            u32 cc = 0;
            if (i < ne) A.entry(i, key, cc);
            if (key < 0) cc = 0;
            i32 f = cc >= 2 ? 1 : 0;
            i32 tb, tp;
            i32 ib = block_incl_scan_i32<BLOCK>(f, sm.wave, tb);
            i32 ip = block_incl_scan_i32<BLOCK>(f ? (i32)cc : 0, sm.wave, tp);
            if (i < ne && key >= 0) {
                u32 h = A.handle(i);
                if (f) {
                    i64 bid = bb + carry_b + ib - 1;
                    A.set_bid(h, (i32)bid);
                    a.boff[bid] = pb + carry_p + ip - (i64)cc;
                    a.bk[bid] = cc;
                    A.set_cnt(h, 0u);  // becomes the fill cursor
                } else {
                    A.set_bid(h, -1);
                }
            }
            carry_b += tb;
            carry_p += tp;
        }
        __syncthreads();
    } else {
        u64 my_start = 0, my_blooms = 0, my_pairs = 0;
        for (i64 i = threadIdx.x; i < ne; i += BLOCK) {
            i32 key;
            u32 c32;
            A.entry(i, key, c32);
            if (key < 0 || c32 < 2) continue;
            u64 cc = c32;
            u64 b = cc * (cc - 1) / 2;
            if (MODE & M_VERTEX) {
                my_start += b;
                atomicAdd((unsigned long long *)&a.sup_label[key], (unsigned long long)b);
                ++t.atomics;
            }
            if (MODE & M_BE_SIZE) {
                my_blooms += 1;
                my_pairs += cc;
            }
        }
        if (MODE & M_VERTEX) {
            u64 tt = block_sum_u64<BLOCK>(my_start, sm.red);
            if (threadIdx.x == 0 && tt) {
                atomicAdd((unsigned long long *)&a.sup_label[s], (unsigned long long)tt);
                ++t.atomics;
            }
        }
        if (MODE & M_BE_SIZE) {
            u64 tb = block_sum_u64<BLOCK>(my_blooms, sm.red);
            u64 tp = block_sum_u64<BLOCK>(my_pairs, sm.red);
            if (threadIdx.x == 0) {
                a.bcnt[s] = (i64)tb;
                a.pcnt[s] = (i64)tp;
            }
        }
        __syncthreads();
    }

    if (MODE & (M_VERTEX | M_EDGE | M_BE_FILL)) {
        sm.agg[threadIdx.x] = 0;
        __syncthreads();
        for_each_wedge<BLOCK>(a, s, sm,
            [&](int seg, i64 jmid, i32 last, i64 pos) {
                u32 h = A.find(last);
                u64 cc;
                if (MODE & M_BE_FILL) {
                    i32 bid = A.bid(h);
                    if (bid < 0) return;
                    // written by this workgroup's epilogue: read coherently
                    cc = ld_coherent(&a.bk[bid]);
                    u32 slot = A.inc(h);
                    i64 p = ld_coherent(&a.boff[bid]) + slot;
                    a.bedge[2 * p] = a.leid[jmid];     // (start, mid)
                    a.bedge[2 * p + 1] = a.leid[pos];  // (mid, last)
                    a.pbloom[p] = bid;
                } else {
                    cc = A.cnt(h);
                    if (cc < 2) return;
                }
                atomicAdd((unsigned long long *)&sm.agg[seg], (unsigned long long)(cc - 1));
                if (MODE & (M_EDGE | M_BE_FILL)) {
                    atomicAdd((unsigned long long *)&a.sup_edge[a.leid[pos]], (unsigned long long)(cc - 1));
                    ++t.atomics;
                }
            },
            [&](i64 cb) {
                u64 g = sm.agg[threadIdx.x];
                if (g) {
                    i64 j = cb + threadIdx.x;
                    if (MODE & M_VERTEX) {
                        atomicAdd((unsigned long long *)&a.sup_label[a.ladj[j]], (unsigned long long)g);
                        ++t.atomics;
                    }
                    if (MODE & (M_EDGE | M_BE_FILL)) {
                        atomicAdd((unsigned long long *)&a.sup_edge[a.leid[j]], (unsigned long long)g);
                        ++t.atomics;
                    }
                    sm.agg[threadIdx.x] = 0;
                }
            });
    }
}

// ------------------------------------------------------------------ kernels

template <int BLOCK, int LOGCAP, int MODE>
__global__ __launch_bounds__(BLOCK) void k_count_hash(CountArgs a) {
    constexpr int CAP = 1 << LOGCAP;
    __shared__ i32 s_keys[CAP];
    __shared__ u32 s_vals[CAP];
    __shared__ i32 s_bids[(MODE & M_BE_FILL) ? CAP : 1];
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ u64 s_agg[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_red[BLOCK / WAVE];
    __shared__ i32 s_item;
    __shared__ i64 s_bcast[1];
    ChunkSmem sm{s_pre, s_moff, s_agg, s_wave, s_red, s_bcast};
    LdsAcc A;
    A.keys = s_keys;
    A.vals = s_vals;
    A.bids = s_bids;
    Tally tl;
    for (;;) {
        if (threadIdx.x == 0) s_item = (i32)atomicAdd(a.next, 1u);
        __syncthreads();
        const i32 item = s_item;
        __syncthreads();
        if (item >= a.nstarts) break;
        const i32 s = a.starts[item];
        // capacity: a power of two at least twice the start's wedge count
        const i64 ws = a.wsum[s];
        int logcap = 6;
        while ((i64(1) << logcap) < 2 * ws && logcap < LOGCAP) ++logcap;
        A.init(logcap, threadIdx.x, BLOCK);
        __syncthreads();
        process_start<BLOCK, MODE>(a, s, A, sm, tl);
        __syncthreads();
    }
    tl.flush(a.kc, a.wedges);
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_count_dense(CountArgs a) {
    // one workgroup per HBM counter slice (the slices bound the grid), so the
    // workgroup is wide: 16 waves per CU hide the scattered counter latency
    constexpr int BLOCK = 1024;
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ u64 s_agg[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_red[BLOCK / WAVE];
    __shared__ i32 s_item;
    __shared__ i64 s_bcast[1];
    ChunkSmem sm{s_pre, s_moff, s_agg, s_wave, s_red, s_bcast};
    DenseAcc A;
    A.c = a.dcnt + (i64)blockIdx.x * a.n;
    A.bids = a.dbid ? a.dbid + (i64)blockIdx.x * a.n : nullptr;
    A.touch = a.dtouch + (i64)blockIdx.x * a.n;
    A.ntouch = a.dntouch + blockIdx.x;
    Tally tl;
    for (;;) {
        if (threadIdx.x == 0) s_item = (i32)atomicAdd(a.next, 1u);
        __syncthreads();
        const i32 item = s_item;
        __syncthreads();
        if (item >= a.nstarts) break;
        const i32 s = a.starts[item];
        process_start<BLOCK, MODE>(a, s, A, sm, tl);
        __syncthreads();
        A.reset(threadIdx.x, BLOCK);
    }
    tl.flush(a.kc, a.wedges);
}

// Large starts of the vertex-count modes, by key tiles.  The lasts of start s
// have smaller labels than s, and the largest starts are the highest-priority
// (smallest-label) vertices, so the keys [0, s) of a large start are covered
// by few tiles of CT = 2^15 consecutive labels (one for every start below
// 2^15).  A work item is one (start, tile) pair: the run of every mid's
// prefix inside the tile is found by binary search (no search when the tile
// is the whole key space), the wedge counts go to dense LDS counters (one u32
// per key, packed (all mids) + 2^16 (hub mids) in the one-side mode) with a
// touched-word bitmap, and the epilogue and second pass are those of the
// hash kernels restricted to the tile's lasts.  Tiles split the lasts, so
// the per-tile contributions of the start, its lasts and its mids add up to
// the per-start ones.
constexpr int CT_LOG = 15;

// tiles of every large start and their exclusive prefix (one workgroup)
__global__ __launch_bounds__(1024) void k_count_tiles(const i32 *starts, u32 nstarts, u32 *off, u32 *total) {
    __shared__ i32 s_wave[1024 / WAVE];
    u32 carry = 0;
    for (u32 base = 0; base < nstarts; base += 1024) {
        const u32 i = base + threadIdx.x;
        i32 r = 0;
        if (i < nstarts) r = (starts[i] + (1 << CT_LOG) - 1) >> CT_LOG;
        i32 tot;
        const i32 incl = block_incl_scan_i32<1024>(r, s_wave, tot);
        if (i < nstarts) off[i] = carry + (u32)(incl - r);
        carry += (u32)tot;
    }
    if (threadIdx.x == 0) {
        off[nstarts] = carry;
        *total = carry;
    }
}

template <int MODE>
__global__ __launch_bounds__(512) void k_count_tiled(CountArgs a, const u32 *off, const u32 *total) {
    constexpr int BLOCK = 512;
    constexpr int CT = 1 << CT_LOG;
    constexpr bool XS = (MODE & M_XSIDE) != 0;
    __shared__ u32 cnt[CT];
    __shared__ u32 bm[CT / 32];
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ u64 s_agg[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_red[BLOCK / WAVE];
    __shared__ u32 s_item;
    for (int i = threadIdx.x; i < CT; i += BLOCK) cnt[i] = 0;
    for (int i = threadIdx.x; i < CT / 32; i += BLOCK) bm[i] = 0;
    const u32 n = *total;
    const u32 ns = a.nstarts;
    Tally tl;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.next, 1u);
        __syncthreads();
        const u32 item = s_item;
        __syncthreads();
        if (item >= n) break;
        u32 lo = 0, hi = ns - 1;
        while (lo < hi) {
            const u32 md = (lo + hi + 1) >> 1;
            if (off[md] <= item) lo = md; else hi = md - 1;
        }
        const i32 s = a.starts[lo];
        const i32 t = (i32)(item - off[lo]);
        const i32 r0 = t << CT_LOG;
        const i32 r1 = r0 + CT < s ? r0 + CT : s;
        const bool whole = r0 == 0 && r1 == s;
        const unsigned char sc = XS ? a.lclass[s] : (unsigned char)0;
        const i64 jb = a.loff[s], je = a.loff[s + 1];
        if (threadIdx.x == 0 && t == 0) {
            tl.segments += (u64)(je - jb);
            tl.items += 1;
        }
        // the wedges of one chunk of mids restricted to the tile; fn(seg, jmid, last, pos)
        auto walk = [&](auto fn, auto chunk_end) {
            for (i64 cb = jb; cb < je; cb += BLOCK) {
                const i64 j = cb + threadIdx.x;
                i32 pl = 0;
                i64 moff = 0;
                if (j < je) {
                    const i32 mid = a.ladj[j];
                    i32 len = a.lpl[j];
                    if (a.alive && !a.alive[mid]) len = 0;
                    const i64 mb = a.loff[mid];
                    i64 b0 = mb, e0 = mb + len;
                    if (!whole && len) {
                        i64 l2 = mb, h2 = e0;
                        while (l2 < h2) {
                            const i64 md = (l2 + h2) >> 1;
                            if (a.ladj[md] < r0) l2 = md + 1; else h2 = md;
                        }
                        b0 = l2;
                        h2 = e0;
                        while (l2 < h2) {
                            const i64 md = (l2 + h2) >> 1;
                            if (a.ladj[md] < r1) l2 = md + 1; else h2 = md;
                        }
                        e0 = l2;
                    }
                    pl = (i32)(e0 - b0);
                    moff = b0;
                }
                i32 tot;
                const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                s_pre[threadIdx.x] = incl;
                s_moff[threadIdx.x] = moff;
                __syncthreads();
                const int last_seg = (je - cb < BLOCK ? (int)(je - cb) : BLOCK) - 1;
                for (i32 kb = 0; kb < tot; kb += CR_UNR * BLOCK)
                    chunk_run<CR_UNR>(a.ladj, s_pre, s_moff, last_seg, kb + (i32)threadIdx.x * CR_UNR, tot,
                                      [&](int seg, i64 pos, i32 last) {
                                          if (a.alive && !a.alive[last]) return;
                                          fn(seg, cb + seg, last, pos);
                                      });
                __syncthreads();
                chunk_end(cb);
                __syncthreads();
            }
        };
        // pass 1: wedge counts per last of the tile
        walk(
            [&](int, i64 jmid, i32 last, i64) {
                u32 inc = 1u;
                if (XS && sc == LC_Y && a.lclass[a.ladj[jmid]] == LC_XHUB) inc = 0x10001u;
                const u32 o = (u32)(last - r0);
                if (atomicAdd(&cnt[o], inc) == 0u) atomicOr(&bm[o >> 5], 1u << (o & 31));
                ++tl.wedges;
            },
            [&](i64) {});
        const bool ends = !XS || sc != LC_Y;  // start and lasts get C(c, 2)
        const bool mids = !XS || sc == LC_Y;  // mids get their shares
        if (ends) {
            u64 my_start = 0;
            const i32 nbw = ((r1 - r0) + 31) >> 5;
            for (i32 bw = threadIdx.x; bw < nbw; bw += BLOCK) {
                u32 bits = bm[bw];
                while (bits) {
                    const i32 o = bw * 32 + (__ffs(bits) - 1);
                    bits &= bits - 1;
                    const u64 cc = XS ? (cnt[o] & 0xFFFFu) : cnt[o];
                    if (cc < 2) continue;
                    const u64 b = cc * (cc - 1) / 2;
                    my_start += b;
                    atomicAdd((unsigned long long *)&a.sup_label[r0 + o], (unsigned long long)b);
                    ++tl.atomics;
                }
            }
            const u64 tt = block_sum_u64<BLOCK>(my_start, s_red);
            if (threadIdx.x == 0 && tt) {
                atomicAdd((unsigned long long *)&a.sup_label[s], (unsigned long long)tt);
                ++tl.atomics;
            }
            __syncthreads();
        }
        if (mids) {
            s_agg[threadIdx.x] = 0;
            __syncthreads();
            walk(
                [&](int seg, i64 jmid, i32 last, i64) {
                    const u32 v = cnt[last - r0];
                    u64 share;
                    if (XS) {
                        const u64 cc = v & 0xFFFFu;
                        if (cc < 2) return;
                        const u64 hub = v >> 16;
                        share = a.lclass[a.ladj[jmid]] == LC_XHUB ? cc - hub : cc - 1;
                    } else {
                        if (v < 2) return;
                        share = (u64)v - 1;
                    }
                    if (share) atomicAdd((unsigned long long *)&s_agg[seg], (unsigned long long)share);
                },
                [&](i64 cb) {
                    const u64 g = s_agg[threadIdx.x];
                    if (g) {
                        atomicAdd((unsigned long long *)&a.sup_label[a.ladj[cb + threadIdx.x]], (unsigned long long)g);
                        ++tl.atomics;
                        s_agg[threadIdx.x] = 0;
                    }
                });
        }
        // clear the touched counters
        const i32 nbw = ((r1 - r0) + 31) >> 5;
        for (i32 bw = threadIdx.x; bw < nbw; bw += BLOCK) {
            u32 bits = bm[bw];
            if (!bits) continue;
            bm[bw] = 0;
            while (bits) {
                cnt[bw * 32 + (__ffs(bits) - 1)] = 0;
                bits &= bits - 1;
            }
        }
        __syncthreads();
    }
    tl.flush(a.kc, a.wedges);
}

// ------------------------------------------------------------------ binning

constexpr i64 SMALL_W = 512, MEDIUM_W = 4096;

// Large starts go to the key-tile kernel (bin 2) when the vertex-count modes
// run and they have at least TILE_MIN_W wedges per tile of their keys on
// average, else to the HBM-counter kernel (bin 3).
constexpr i64 TILE_MIN_W = 2048;

__global__ void k_bin_starts(const i64 *wsum, const unsigned char *lclass, const unsigned char *alive, i64 n, i32 *lists,
                             u32 *counts, int tiles_ok) {
    // lists: [4][n]; counts: [4]; one atomic per wave and bin
    const i64 stride = (i64)gridDim.x * blockDim.x;
    const i64 nn = (n + WAVE - 1) / WAVE * WAVE;
    for (i64 s = blockIdx.x * (i64)blockDim.x + threadIdx.x; s < nn; s += stride) {
        int b = -1;
        if (s < n) {
            const i64 w = wsum[s];
            const bool skip = w == 0 || (alive && !alive[s]) || (lclass && lclass[s] == LC_XHUB);
            if (!skip) {
                if (w <= SMALL_W) b = 0;
                else if (w <= MEDIUM_W) b = 1;
                else {
                    const i64 tiles = (s + (i64(1) << CT_LOG) - 1) >> CT_LOG;
                    b = tiles_ok && w >= tiles * TILE_MIN_W ? 2 : 3;
                }
            }
        }
        for (int k = 0; k < 4; ++k) {
            const u32 p = wave_append(&counts[k], b == k);
            if (b == k) lists[(i64)k * n + p] = (i32)s;
        }
    }
}

static int gridN(i64 n) {
    i64 g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

struct Bins {
    i32 *lists;
    u32 cnt[4];
};

static Bins bin_starts(Ctx &c, const DevGraph &G, const unsigned char *alive, const unsigned char *lclass, bool tiles_ok) {
    Bins b;
    b.lists = c.alloc<i32>(4 * G.n);
    u32 *counts = c.alloc<u32>(4);
    PBNG_HIP(hipMemsetAsync(counts, 0, 4 * sizeof(u32), c.stream));
    if (G.n) {
        hipLaunchKernelGGL(k_bin_starts, dim3(gridN(G.n)), dim3(256), 0, c.stream, (const i64 *)G.wsum, lclass, alive, G.n,
                           b.lists, counts, tiles_ok ? 1 : 0);
        PBNG_LAUNCH_CHECK();
    }
    PBNG_HIP(hipMemcpyAsync(b.cnt, counts, 4 * sizeof(u32), hipMemcpyDeviceToHost, c.stream));
    PBNG_HIP(hipStreamSynchronize(c.stream));
    return b;
}

template <int MODE>
static void launch_all(Ctx &c, const DevGraph &G, CountArgs a, const Bins &b) {
    u32 *next = c.alloc<u32>(4);
    PBNG_HIP(hipMemsetAsync(next, 0, 4 * sizeof(u32), c.stream));
    a.kc = c.kctr + PBNG_K_COUNT;
    int slots = (int)std::min<i64>(b.cnt[3], (i64)c.num_cu);
    if (b.cnt[3] && c.arena.fixed_base) {
        // fixed scratch: as many HBM counter slices as half the room left holds
        const size_t per = (size_t)std::max<i64>(G.n, 1) * ((MODE & M_BE_FILL) ? 12 : 8);
        slots = (int)std::max<size_t>(1, std::min<size_t>((size_t)slots, c.arena.fixed_left() / 2 / per));
    }
    if (b.cnt[3]) {
        a.dcnt = c.alloc<u32>((i64)slots * G.n);
        a.dtouch = c.alloc<i32>((i64)slots * G.n);
        a.dbid = (MODE & M_BE_FILL) ? c.alloc<i32>((i64)slots * G.n) : nullptr;
        a.dntouch = c.alloc<u32>(slots);
        PBNG_HIP(hipMemsetAsync(a.dcnt, 0, sizeof(u32) * slots * G.n, c.stream));
        PBNG_HIP(hipMemsetAsync(a.dntouch, 0, sizeof(u32) * slots, c.stream));
    }
    c.kbegin(PBNG_K_COUNT);
    // large starts first: they are the long tail
    if (b.cnt[3]) {
        a.starts = b.lists + 3 * G.n;
        a.nstarts = b.cnt[3];
        a.next = next + 3;
        hipLaunchKernelGGL(k_count_dense<MODE>, dim3(slots), dim3(1024), 0, c.stream, a);
        PBNG_LAUNCH_CHECK();
    }
    if constexpr (MODE == M_XSIDE || MODE == M_VERTEX) {
        if (b.cnt[2]) {
            a.starts = b.lists + 2 * G.n;
            a.nstarts = b.cnt[2];
            a.next = next + 2;
            u32 *toff = c.alloc<u32>((i64)b.cnt[2] + 1);
            u32 *ttot = c.alloc<u32>(1);
            hipLaunchKernelGGL(k_count_tiles, dim3(1), dim3(1024), 0, c.stream, (const i32 *)a.starts, (u32)b.cnt[2], toff,
                               ttot);
            hipLaunchKernelGGL(k_count_tiled<MODE>, dim3(c.num_cu), dim3(512), 0, c.stream, a, (const u32 *)toff,
                               (const u32 *)ttot);
            PBNG_LAUNCH_CHECK();
        }
    }
    if (b.cnt[1]) {
        a.starts = b.lists + G.n;
        a.nstarts = b.cnt[1];
        a.next = next + 1;
        int grid = (int)std::min<i64>(b.cnt[1], (i64)c.num_cu * 2);
        hipLaunchKernelGGL((k_count_hash<512, 13, MODE>), dim3(grid), dim3(512), 0, c.stream, a);
        PBNG_LAUNCH_CHECK();
    }
    if (b.cnt[0]) {
        a.starts = b.lists;
        a.nstarts = b.cnt[0];
        a.next = next;
        int grid = (int)std::min<i64>(b.cnt[0], (i64)c.num_cu * 16);
        hipLaunchKernelGGL((k_count_hash<64, 10, MODE>), dim3(grid), dim3(64), 0, c.stream, a);
        PBNG_LAUNCH_CHECK();
    }
    c.kend(PBNG_K_COUNT);
}

static CountArgs base_args(const DevGraph &G) {
    CountArgs a{};
    a.loff = G.loff;
    a.ladj = G.ladj;
    a.leid = G.leid;
    a.lpl = G.lpl;
    a.wsum = G.wsum;
    a.n = G.n;
    return a;
}

u64 count_pass(Ctx &c, const DevGraph &G, u64 *sup_label, u64 *sup_edge, const unsigned char *alive) {
    CountArgs a = base_args(G);
    a.alive = alive;
    a.sup_label = sup_label;
    a.sup_edge = sup_edge;
    a.wedges = c.alloc<u64>(1);
    PBNG_HIP(hipMemsetAsync(a.wedges, 0, sizeof(u64), c.stream));
    if (sup_label) PBNG_HIP(hipMemsetAsync(sup_label, 0, sizeof(u64) * (G.n ? G.n : 1), c.stream));
    if (sup_edge) PBNG_HIP(hipMemsetAsync(sup_edge, 0, sizeof(u64) * (G.m ? G.m : 1), c.stream));
    Bins b = bin_starts(c, G, alive, nullptr, sup_label && !sup_edge);
    if (sup_label && sup_edge) launch_all<M_VERTEX | M_EDGE>(c, G, a, b);
    else if (sup_label) launch_all<M_VERTEX>(c, G, a, b);
    else if (sup_edge) launch_all<M_EDGE>(c, G, a, b);
    return read_scalar<u64>(c, a.wedges);
}

u64 count_pass_xside(Ctx &c, const DevGraph &G, u64 *sup_label, const unsigned char *lclass) {
    CountArgs a = base_args(G);
    a.lclass = lclass;
    a.sup_label = sup_label;
    a.wedges = c.alloc<u64>(1);
    PBNG_HIP(hipMemsetAsync(a.wedges, 0, sizeof(u64), c.stream));
    PBNG_HIP(hipMemsetAsync(sup_label, 0, sizeof(u64) * (G.n ? G.n : 1), c.stream));
    Bins b = bin_starts(c, G, nullptr, lclass, true);
    launch_all<M_XSIDE>(c, G, a, b);
    return read_scalar<u64>(c, a.wedges);
}

void count_butterflies(Ctx &c, const DevGraph &G, const CountOut &out, const pbng_opts &) {
    u64 w = count_pass(c, G, out.sup_label, out.sup_edge, nullptr);
    c.stats.wedges_count += w;
    c.stats.wedges += w;
}

// ------------------------------------------------------------------ gather

__global__ void k_gather_side(const u64 *sup_label, const i32 *label, i64 off, i64 cnt, u64 *out) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < cnt; i += (i64)gridDim.x * blockDim.x)
        out[i] = sup_label[label[off + i]];
}

void gather_side(Ctx &c, const DevGraph &G, const u64 *sup_label, int side, u64 *out) {
    i64 off = side == 0 ? 0 : G.n_u;
    i64 cnt = side == 0 ? G.n_u : G.n_v;
    if (!cnt) return;
    hipLaunchKernelGGL(k_gather_side, dim3(gridN(cnt)), dim3(256), 0, c.stream, sup_label, (const i32 *)G.label, off, cnt, out);
    PBNG_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ BE-Index

__global__ void k_edge_link_count(const i32 *bedge, i64 npairs, u32 *ecnt) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < npairs; p += (i64)gridDim.x * blockDim.x) {
        atomicAdd(&ecnt[bedge[2 * p]], 1u);
        atomicAdd(&ecnt[bedge[2 * p + 1]], 1u);
    }
}

__global__ void k_u32_to_i64(const u32 *a, i64 n, i64 *b) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) b[i] = a[i];
}

__global__ void k_edge_link_fill(const i32 *bedge, const i32 *pbloom, i64 npairs, i64 *cursor, i32 *ebloom, i32 *etwin) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < npairs; p += (i64)gridDim.x * blockDim.x) {
        i32 e1 = bedge[2 * p], e2 = bedge[2 * p + 1], b = pbloom[p];
        i64 q1 = atomicAdd((unsigned long long *)&cursor[e1], 1ull);
        ebloom[q1] = b;
        etwin[q1] = e2;
        i64 q2 = atomicAdd((unsigned long long *)&cursor[e2], 1ull);
        ebloom[q2] = b;
        etwin[q2] = e1;
    }
}

void build_be_index(Ctx &c, const DevGraph &G, BEIndex &I, u64 *sup_edge) {
    const i64 n = G.n, m = G.m;
    CountArgs a = base_args(G);
    a.wedges = c.alloc<u64>(1);
    PBNG_HIP(hipMemsetAsync(a.wedges, 0, sizeof(u64), c.stream));
    Bins b = bin_starts(c, G, nullptr, nullptr, false);
    // sizes
    a.bcnt = c.alloc<i64>(n);
    a.pcnt = c.alloc<i64>(n);
    PBNG_HIP(hipMemsetAsync(a.bcnt, 0, sizeof(i64) * (n ? n : 1), c.stream));
    PBNG_HIP(hipMemsetAsync(a.pcnt, 0, sizeof(i64) * (n ? n : 1), c.stream));
    launch_all<M_BE_SIZE>(c, G, a, b);
    i64 *bbase = c.alloc<i64>(n + 1);
    i64 *pbase = c.alloc<i64>(n + 1);
    exclusive_scan<i64>(c, a.bcnt, bbase, n);
    exclusive_scan<i64>(c, a.pcnt, pbase, n);
    I.nblooms = read_scalar<i64>(c, bbase + n);
    I.npairs = read_scalar<i64>(c, pbase + n);
    if (I.nblooms >= (i64(1) << 31) || 2 * I.npairs >= (i64(1) << 40))
        throw Error(PBNG_E_OVERFLOW, "BE-Index larger than the index widths");
    I.boff = c.alloc<i64>(I.nblooms + 1);
    I.bk = c.alloc<u32>(I.nblooms);
    I.bedge = c.alloc<i32>(2 * I.npairs);
    i32 *pbloom = c.alloc<i32>(I.npairs);
    I.pbloom = pbloom;
    // fill (also the per-edge supports)
    a.bbase = bbase;
    a.pbase = pbase;
    a.boff = I.boff;
    a.bk = I.bk;
    a.bedge = I.bedge;
    a.pbloom = pbloom;
    a.sup_edge = sup_edge;
    PBNG_HIP(hipMemsetAsync(sup_edge, 0, sizeof(u64) * (m ? m : 1), c.stream));
    launch_all<M_BE_FILL>(c, G, a, b);
    PBNG_HIP(hipMemcpyAsync(I.boff + I.nblooms, &I.npairs, sizeof(i64), hipMemcpyHostToDevice, c.stream));
    // edge-major links
    u32 *ecnt = c.alloc<u32>(m);
    i64 *ecnt64 = c.alloc<i64>(m);
    PBNG_HIP(hipMemsetAsync(ecnt, 0, sizeof(u32) * (m ? m : 1), c.stream));
    if (I.npairs) {
        hipLaunchKernelGGL(k_edge_link_count, dim3(gridN(I.npairs)), dim3(256), 0, c.stream, (const i32 *)I.bedge, I.npairs, ecnt);
        PBNG_LAUNCH_CHECK();
    }
    if (m) {
        hipLaunchKernelGGL(k_u32_to_i64, dim3(gridN(m)), dim3(256), 0, c.stream, (const u32 *)ecnt, m, ecnt64);
        PBNG_LAUNCH_CHECK();
    }
    I.eoff = c.alloc<i64>(m + 1);
    exclusive_scan<i64>(c, ecnt64, I.eoff, m);
    i64 *cursor = c.alloc<i64>(m);
    if (m) PBNG_HIP(hipMemcpyAsync(cursor, I.eoff, sizeof(i64) * m, hipMemcpyDeviceToDevice, c.stream));
    I.ebloom = c.alloc<i32>(2 * I.npairs);
    I.etwin = c.alloc<i32>(2 * I.npairs);
    if (I.npairs) {
        hipLaunchKernelGGL(k_edge_link_fill, dim3(gridN(I.npairs)), dim3(256), 0, c.stream, (const i32 *)I.bedge,
                           (const i32 *)pbloom, I.npairs, cursor, I.ebloom, I.etwin);
        PBNG_LAUNCH_CHECK();
    }
    u64 w = read_scalar<u64>(c, a.wedges);
    c.stats.wedges_count += w;
    c.stats.wedges += w;
    c.stats.blooms = I.nblooms;
    c.stats.bloom_pairs = I.npairs;
}

}  // namespace pbng
