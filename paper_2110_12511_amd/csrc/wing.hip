// Wing decomposition by two-phase peeling with the BE-Index (Sections 2.3,
// 3.3; Algorithms 3-6).
//
// Entities are edges; a bloom B holds k_B twin pairs (its bloom number), and
// every butterfly of G is one pair of pairs of exactly one bloom.
//
// Coarse-grained phase, one round over an active edge set S (Algorithm 6,
// batched):
//   links kernel  - for each active e and each of its live blooms B with twin
//                   t (when both twins are active only the one with the
//                   larger edge id acts, the tie rule of Algorithm 4): t, if
//                   alive, loses k_B - 1 (all of its butterflies in B; k_B is
//                   read before any bloom changes), and count[B] grows by one;
//   blooms kernel - for each touched bloom: k_B -= count[B]; pairs holding an
//                   active edge are dropped from B's pair list (dynamic graph
//                   update, Section 5.2); every edge of a surviving pair loses
//                   count[B] (one butterfly per dropped pair).
// Supports that cross below the bound form the next active set.  Plain
// atomic subtraction is enough: an alive edge's support is its exact count
// of remaining butterflies and never goes below it.
//
// Fine-grained phase (Algorithm 5): a pair of twins (e1, e2) belongs to
// partition min(p(e1), p(e2)) only; there its bloom instance has bloom number
// k_B(I_i) = number of B's pairs whose minimum partition is >= i, and its
// links are the pair's edges that lie in partition i.  Each partition is
// peeled alone from its initialisation vector, level by level (all alive
// edges at the minimum support at once; the same twin rule decides inside a
// level; max(level, .) clamps of one level commute), in one persistent
// kernel whose workgroups pop partitions in decreasing work order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "dev_common.h"
#include "pbng_internal.h"

namespace pbng {

enum : unsigned char { WS_ALIVE = 0, WS_ACTIVE = 1, WS_PEELED = 2 };

struct WingCtl {
    u64 bound;
    u64 s;
    u64 est_init;
    u64 est_final;
    double scale;
    u32 nF, nF2;
    u32 ntouch;     // blooms touched this round
    u32 pad;
    u64 updates;    // support updates
    u64 links;      // links walked
    i32 pid;        // partition being built
    u32 pad2;
    u64 rounds;     // rounds that had active edges
    i64 alive;      // edges neither peeled nor active
};

// rounds per replay of the captured coarse-grained round graph (even, so the
// two active-set buffers are back in place after a replay)
constexpr int W_GRAPH_K = 4;

// ------------------------------------------------------------------ CD kernels

__global__ void w_frontier(unsigned char *st, const u64 *sup, u64 *init, i32 *part, i64 m, WingCtl *ctl, i32 pid,
                           i32 *F) {
    const u64 B = ctl->bound;
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        if (st[e] != WS_ALIVE) continue;
        const u64 s = sup[e];
        init[e] = s;
        if (s < B) {
            st[e] = WS_ACTIVE;
            part[e] = pid;
            u32 p = atomicAdd(&ctl->nF, 1u);
            F[p] = (i32)e;
        }
    }
}

__device__ __forceinline__ void w_dec(u64 *sup, i32 e, u64 d, u64 B, i32 *F2, u32 *nF2) {
    const u64 old = atomicAdd((unsigned long long *)&sup[e], (unsigned long long)(0ull - d));
    if (old >= B && old - d < B) {
        u32 p = atomicAdd(nF2, 1u);
        F2[p] = e;
    }
}

// One wave per active edge, lanes over its links.
__global__ void w_links(const i32 *F, const u32 *nF, const i64 *eoff, const i32 *ebloom, const i32 *etwin,
                        const unsigned char *st, const u32 *bk, u32 *bcount, i32 *touched, u64 *sup, WingCtl *ctl,
                        i32 *F2, KCounters *kc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *nF;
    const u64 B = ctl->bound;
    Tally t;
    u64 upd = 0;
    for (i64 i = wave; i < n; i += nwaves) {
        const i32 e = F[i];
        for (i64 q = eoff[e] + lane; q < eoff[e + 1]; q += WAVE) {
            ++t.wedges;
            const i32 et = etwin[q];
            const unsigned char s = st[et];
            if (s == WS_PEELED) continue;           // pair dropped earlier
            if (s == WS_ACTIVE && et > e) continue;  // the larger twin acts
            const i32 b = ebloom[q];
            if (s == WS_ALIVE) {
                const u32 kb = bk[b];
                const u64 d = kb > 1 ? (u64)kb - 1 : 0;
                if (d) {
                    w_dec(sup, et, d, B, F2, &ctl->nF2);
                    ++upd;
                }
            }
            if (atomicAdd(&bcount[b], 1u) == 0) {
                u32 p = atomicAdd(&ctl->ntouch, 1u);
                touched[p] = b;
                ++t.segments;
            }
        }
    }
    t.atomics = upd;
    for (int d = WAVE / 2; d > 0; d >>= 1) upd += __shfl_down(upd, d, WAVE);
    if (lane == 0 && upd) atomicAdd((unsigned long long *)&ctl->updates, (unsigned long long)upd);
    u64 lk = t.wedges;
    for (int d = WAVE / 2; d > 0; d >>= 1) lk += __shfl_down(lk, d, WAVE);
    if (lane == 0 && lk) atomicAdd((unsigned long long *)&ctl->links, (unsigned long long)lk);
    t.flush(kc, nullptr);
}

// Unbatched form of the round (the PBNG-- ablation, Section 6.3.2): the
// twin updates and bloom counts of w_links, but every acting link then walks
// its bloom itself and takes one butterfly from both edges of every alive
// pair, instead of each touched bloom subtracting its count once (w_blooms
// then only drops pairs and lowers k_B).  The totals per edge are the same,
// count[B] per bloom; the work is one bloom walk per peeled pair.  One wave
// per active edge: lanes evaluate 64 links, then the wave walks the bloom of
// each acting one.
__global__ void w_links_each(const i32 *F, const u32 *nF, const i64 *eoff, const i32 *ebloom, const i32 *etwin,
                             const unsigned char *st, const u32 *bk, u32 *bcount, i32 *touched, const i64 *boff,
                             const u32 *blen, const i32 *bedge, u64 *sup, WingCtl *ctl, i32 *F2, KCounters *kc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *nF;
    const u64 B = ctl->bound;
    Tally t;
    u64 upd = 0;
    for (i64 i = wave; i < n; i += nwaves) {
        const i32 e = F[i];
        const i64 q1 = eoff[e + 1];
        for (i64 q0 = eoff[e]; q0 < q1; q0 += WAVE) {
            const i64 q = q0 + lane;
            bool act = false;
            i32 b = -1;
            if (q < q1) {
                ++t.wedges;
                const i32 et = etwin[q];
                const unsigned char s = st[et];
                // pair dropped earlier, or both active and the larger twin acts
                if (s != WS_PEELED && !(s == WS_ACTIVE && et > e)) {
                    act = true;
                    b = ebloom[q];
                    if (s == WS_ALIVE) {
                        const u32 kb = bk[b];
                        const u64 d = kb > 1 ? (u64)kb - 1 : 0;
                        if (d) {
                            w_dec(sup, et, d, B, F2, &ctl->nF2);
                            ++upd;
                        }
                    }
                    if (atomicAdd(&bcount[b], 1u) == 0) {
                        u32 p = atomicAdd(&ctl->ntouch, 1u);
                        touched[p] = b;
                        ++t.segments;
                    }
                }
            }
            u64 bal = __ballot(act);
            while (bal) {
                const int k = __builtin_ctzll(bal);
                bal &= bal - 1;
                const i32 bb = __shfl(b, k, WAVE);
                const i64 base = boff[bb];
                const i32 len = (i32)blen[bb];
                for (i32 pp = lane; pp < len; pp += WAVE) {
                    const i32 e1 = bedge[2 * (base + pp)], e2 = bedge[2 * (base + pp) + 1];
                    if (st[e1] == WS_ALIVE && st[e2] == WS_ALIVE) {
                        w_dec(sup, e1, 1, B, F2, &ctl->nF2);
                        w_dec(sup, e2, 1, B, F2, &ctl->nF2);
                        upd += 2;
                    }
                }
            }
        }
    }
    t.atomics = upd;
    for (int d = WAVE / 2; d > 0; d >>= 1) upd += __shfl_down(upd, d, WAVE);
    if (lane == 0 && upd) atomicAdd((unsigned long long *)&ctl->updates, (unsigned long long)upd);
    u64 lk = t.wedges;
    for (int d = WAVE / 2; d > 0; d >>= 1) lk += __shfl_down(lk, d, WAVE);
    if (lane == 0 && lk) atomicAdd((unsigned long long *)&ctl->links, (unsigned long long)lk);
    t.flush(kc, nullptr);
}

// One wave per touched bloom: drop pairs with a non-alive edge (in place,
// order kept), subtract count[B] from both edges of every surviving pair
// (unless the round's links already did, decrement = 0).
__global__ void w_blooms(const i32 *touched, const u32 *ntouch, const i64 *boff, u32 *blen, u32 *bk, u32 *bcount,
                         i32 *bedge, const unsigned char *st, u64 *sup, WingCtl *ctl, i32 *F2, int dynamic, int decrement,
                         KCounters *kc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 n = *ntouch;
    const u64 B = ctl->bound;
    const u64 lt = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    Tally t;
    u64 upd = 0;
    for (i64 i = wave; i < n; i += nwaves) {
        const i32 b = touched[i];
        const u64 cnt = bcount[b];
        const i64 base = boff[b];
        const i32 len = (i32)blen[b];
        i32 out = 0;
        for (i32 k0 = 0; k0 < len; k0 += WAVE) {
            const i32 k = k0 + lane;
            i32 e1 = -1, e2 = -1;
            bool keep = false;
            if (k < len) {
                e1 = bedge[2 * (base + k)];
                e2 = bedge[2 * (base + k) + 1];
                keep = st[e1] == WS_ALIVE && st[e2] == WS_ALIVE;
                t.wedges += 2;
            }
            if (keep && decrement) {
                w_dec(sup, e1, cnt, B, F2, &ctl->nF2);
                w_dec(sup, e2, cnt, B, F2, &ctl->nF2);
                upd += 2;
            }
            if (dynamic) {
                const u64 bal = __ballot(keep);
                if (keep) {
                    const i64 o = base + out + __popcll(bal & lt);
                    bedge[2 * o] = e1;
                    bedge[2 * o + 1] = e2;
                }
                out += __popcll(bal);
            }
        }
        if (lane == 0) {
            if (dynamic) blen[b] = (u32)out;
            bk[b] -= (u32)cnt;
            bcount[b] = 0;
            t.items += 1;
        }
    }
    t.atomics = upd;
    for (int d = WAVE / 2; d > 0; d >>= 1) upd += __shfl_down(upd, d, WAVE);
    if (lane == 0 && upd) atomicAdd((unsigned long long *)&ctl->updates, (unsigned long long)upd);
    t.flush(kc, nullptr);
}

__global__ void w_retire(const i32 *F, const u32 *nF, unsigned char *st, const u64 *init, WingCtl *ctl) {
    const u32 n = *nF;
    u64 s = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const i32 e = F[i];
        st[e] = WS_PEELED;
        s += init[e];
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) s += __shfl_down(s, d, WAVE);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd((unsigned long long *)&ctl->est_final, (unsigned long long)s);
}

__global__ void w_activate(const i32 *F2, const u32 *nF2, unsigned char *st, i32 *part, const WingCtl *ctl) {
    const u32 n = *nF2;
    const i32 pid = ctl->pid;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const i32 e = F2[i];
        st[e] = WS_ACTIVE;
        part[e] = pid;
    }
}

__global__ void w_set_bound(WingCtl *ctl, int last, i32 pid) {
    ctl->bound = last ? ~0ull : ctl->s + 1;
    ctl->nF = 0;
    ctl->nF2 = 0;
    ctl->ntouch = 0;
    ctl->est_final = 0;
    ctl->pid = pid;
}

// the next active set becomes current; the retired edges leave the alive count
__global__ void w_next_round(WingCtl *ctl) {
    if (ctl->nF) {
        ctl->rounds += 1;
        ctl->alive -= (i64)ctl->nF;
    }
    ctl->nF = ctl->nF2;
    ctl->nF2 = 0;
    ctl->ntouch = 0;
}

// alive count after a partition's first active set is drawn
__global__ void w_alive_init(WingCtl *ctl, i64 m) { ctl->alive = m; }

__global__ void w_scale(WingCtl *ctl) {
    const double fin = (double)ctl->est_final;
    ctl->scale = fin > 0 ? (double)ctl->est_init / fin : 1.0;
    if (!(ctl->scale > 0)) ctl->scale = 1.0;
}

__global__ void w_blen_init(const i64 *boff, i64 nb, u32 *blen) {
    for (i64 b = blockIdx.x * (i64)blockDim.x + threadIdx.x; b < nb; b += (i64)gridDim.x * blockDim.x)
        blen[b] = (u32)(boff[b + 1] - boff[b]);
}

__device__ inline u64 w_splitmix(u64 z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void w_minmax(const u64 *sup, const unsigned char *st, i64 m, u64 *mn, u64 *mx) {
    u64 a = ~0ull, b = 0;
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        if (st[e] != WS_ALIVE) continue;
        const u64 s = sup[e];
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

__global__ void w_random_pick(WingCtl *ctl, const u64 *mn, const u64 *mx, u64 seed, int i) {
    const u64 lo = *mn, hi = *mx;
    const u64 span = hi - lo + 1;
    const u64 r = w_splitmix(seed * 1000003ull + (u64)i + 77);
    ctl->s = lo + (span > 1 ? r % (span / 4 + 1) : 0);
}

// ------------------------------------------------------------------ FD preparation

__global__ void w_part_keys(const i32 *part, i64 m, u64 *keys, i32 *vals) {
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        keys[e] = (u64)part[e];
        vals[e] = (i32)e;
    }
}

__global__ void w_u32_to_i64(const u32 *a, i64 n, i64 *b) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) b[i] = a[i];
}

__global__ void w_loc(const i32 *es, const i32 *part, const i64 *epoff, i64 m, i32 *eloc) {
    for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < m; k += (i64)gridDim.x * blockDim.x) {
        const i32 e = es[k];
        eloc[e] = (i32)(k - epoff[part[e]]);
    }
}

// key (bloom, partition of the pair) for the bloom-number suffix counts
__global__ void w_pair_keys_bp(const i32 *bedge, const i32 *pbloom, const i32 *part, i64 np_pairs, i32 np, u64 *keys,
                               i32 *vals) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < np_pairs; p += (i64)gridDim.x * blockDim.x) {
        const i32 a = part[bedge[2 * p]], b = part[bedge[2 * p + 1]];
        const i32 mn = a < b ? a : b;
        keys[p] = (u64)pbloom[p] * (u64)np + (u64)mn;
        vals[p] = (i32)p;
    }
}

// k_B(I_i) for every pair: pairs of B whose minimum partition is >= i
__global__ void w_pair_k(const u64 *skeys, const i32 *svals, const i64 *boff, const i32 *pbloom, i64 np_pairs, u32 *pk) {
    for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < np_pairs; q += (i64)gridDim.x * blockDim.x) {
        const i32 p = svals[q];
        const i32 b = pbloom[p];
        const u64 key = skeys[q];
        i64 lo = boff[b], hi = q;  // first position in B's run with this key
        while (lo < hi) {
            const i64 md = (lo + hi) >> 1;
            if (skeys[md] < key) lo = md + 1; else hi = md;
        }
        pk[p] = (u32)(boff[b + 1] - lo);
    }
}

__global__ void w_pair_keys_pb(const i32 *bedge, const i32 *pbloom, const i32 *part, i64 np_pairs, i64 nblooms, u64 *keys,
                               i32 *vals) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < np_pairs; p += (i64)gridDim.x * blockDim.x) {
        const i32 a = part[bedge[2 * p]], b = part[bedge[2 * p + 1]];
        const i32 mn = a < b ? a : b;
        keys[p] = (u64)mn * (u64)nblooms + (u64)pbloom[p];
        vals[p] = (i32)p;
    }
}

// FD pair arrays in (partition, bloom) order and instance starts
__global__ void w_fd_pairs(const u64 *skeys, const i32 *svals, const i32 *bedge, i64 np_pairs, i32 *fpair, u32 *isstart) {
    for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < np_pairs; q += (i64)gridDim.x * blockDim.x) {
        const i32 p = svals[q];
        fpair[2 * q] = bedge[2 * p];
        fpair[2 * q + 1] = bedge[2 * p + 1];
        isstart[q] = (q == 0 || skeys[q] != skeys[q - 1]) ? 1u : 0u;
    }
}

// instance records: start, length, bloom number; partition of each instance
__global__ void w_fd_instances(const u64 *skeys, const i32 *svals, const u32 *isstart, const u32 *iidx_excl, i64 np_pairs,
                               i64 nblooms, const u32 *pk, i64 *ipstart, u32 *ik, i32 *ipart, u32 *pinst) {
    for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < np_pairs; q += (i64)gridDim.x * blockDim.x) {
        const u32 inst = iidx_excl[q] + isstart[q] - 1;
        pinst[q] = inst;
        if (isstart[q]) {
            ipstart[inst] = q;
            ik[inst] = pk[svals[q]];
            ipart[inst] = (i32)(skeys[q] / (u64)nblooms);
        }
    }
}

__global__ void w_fd_instance_len(const i64 *ipstart, i64 ninst, i64 np_pairs, u32 *iplen) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < ninst; t += (i64)gridDim.x * blockDim.x) {
        const i64 end = t + 1 < ninst ? ipstart[t + 1] : np_pairs;
        iplen[t] = (u32)(end - ipstart[t]);
    }
}

// links of partition edges: count per edge (es order), then fill
__global__ void w_fd_link_count(const i32 *fpair, const u32 *pinst, const i32 *ipart, const i32 *part, const i64 *epoff,
                                const i32 *eloc, i64 np_pairs, u32 *lcnt) {
    for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < np_pairs; q += (i64)gridDim.x * blockDim.x) {
        const i32 i = ipart[pinst[q]];
        for (int h = 0; h < 2; ++h) {
            const i32 e = fpair[2 * q + h];
            if (part[e] == i) atomicAdd(&lcnt[epoff[i] + eloc[e]], 1u);
        }
    }
}

__global__ void w_fd_link_fill(const i32 *fpair, const u32 *pinst, const i32 *ipart, const i32 *part, const i64 *epoff,
                               const i32 *eloc, i64 np_pairs, i64 *lcur, u32 *linst, i32 *ltwin) {
    for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < np_pairs; q += (i64)gridDim.x * blockDim.x) {
        const u32 t = pinst[q];
        const i32 i = ipart[t];
        for (int h = 0; h < 2; ++h) {
            const i32 e = fpair[2 * q + h];
            if (part[e] != i) continue;
            const i64 pos = atomicAdd((unsigned long long *)&lcur[epoff[i] + eloc[e]], 1ull);
            linst[pos] = t;
            ltwin[pos] = fpair[2 * q + (h ^ 1)];
        }
    }
}

__global__ void w_part_first_inst(const i32 *ipart, i64 ninst, i64 *pfirst) {
    // pfirst[i] = first instance of partition i (instances are sorted by partition)
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < ninst; t += (i64)gridDim.x * blockDim.x)
        if (t == 0 || ipart[t] != ipart[t - 1]) pfirst[ipart[t]] = t;
}



__global__ void w_lpt_keys(const u64 *work, i32 np, u64 maxw, u64 *keys, i32 *vals) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < np; p += (i64)gridDim.x * blockDim.x) {
        keys[p] = maxw - work[p];
        vals[p] = (i32)p;
    }
}

__global__ void w_max_u64(const u64 *a, i64 n, u64 *out, u64 *sum) {
    u64 mx = 0, s = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        mx = a[i] > mx ? a[i] : mx;
        s += a[i];
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        u64 o = __shfl_down(mx, d, WAVE);
        mx = o > mx ? o : mx;
        s += __shfl_down(s, d, WAVE);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax((unsigned long long *)out, (unsigned long long)mx);
        if (sum) atomicAdd((unsigned long long *)sum, (unsigned long long)s);
    }
}

// ------------------------------------------------------------------ FD kernel

struct WFdArgs {
    const i32 *es;       // edges grouped by partition
    const i64 *epoff;    // [np+1]
    const i32 *eloc;     // position of an edge inside its partition
    const i32 *part;
    const i64 *loff;     // [m+1] link offsets in es order
    const u32 *linst;    // link -> instance
    const i32 *ltwin;    // link -> twin edge
    const i64 *ipstart;  // instance -> first pair
    u32 *iplen;          // instance -> pairs (pairs of dropped twins are marked)
    u32 *ik;             // instance -> bloom number in its partition
    u32 *icount;         // instance -> pairs dropped this level (zero between levels)
    i32 *fpair;          // FD pairs (2 edge ids)
    const i32 *queue;
    i32 np;
    u32 *head;
    const u64 *init;
    u64 *theta;
    // per-workgroup scratch, stride maxne
    i64 *lsup;
    unsigned char *lst;
    i32 *lbatch;
    u32 *ltouch;
    i64 maxne;
    i64 tstride;         // ltouch stride: most instances of one partition
    u64 *work;           // links + pair visits
    KCounters *kc;
    u32 *levels;         // optional: levels peeled per partition
};

// st: 1 alive, 2 in the current level's batch, 0 peeled
__global__ __launch_bounds__(256) void k_wing_fd(WFdArgs a) {
    constexpr int BLOCK = 256;
    __shared__ i32 s_pre[BLOCK];
    __shared__ i64 s_moff[BLOCK];
    __shared__ i32 s_own[BLOCK];
    __shared__ i32 s_wave[BLOCK / WAVE];
    __shared__ u64 s_red[BLOCK / WAVE];
    __shared__ i32 s_item;
    __shared__ u32 s_cnt[2];
    i64 *lsup = a.lsup + blockIdx.x * a.maxne;
    unsigned char *lst = a.lst + blockIdx.x * a.maxne;
    i32 *lbatch = a.lbatch + blockIdx.x * a.maxne;
    u32 *ltouch = a.ltouch + blockIdx.x * a.tstride;
    u64 work = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = (i32)atomicAdd(a.head, 1u);
        __syncthreads();
        const i32 qi = s_item;
        __syncthreads();
        if (qi >= a.np) break;
        const i32 pid = a.queue[qi];
        const i64 base = a.epoff[pid];
        const i32 ne = (i32)(a.epoff[pid + 1] - base);
        for (i32 k = threadIdx.x; k < ne; k += BLOCK) {
            st_coherent(&lsup[k], (i64)a.init[a.es[base + k]]);
            st_coherent(&lst[k], (unsigned char)1);
        }
        __syncthreads();
        i32 remaining = ne;
        while (remaining > 0) {
            // the minimum alive support and the batch at that level
            u64 mn = ~0ull;
            for (i32 k = threadIdx.x; k < ne; k += BLOCK)
                if (ld_coherent(&lst[k]) == 1) {
                    const u64 s = (u64)ld_coherent((const u64 *)&lsup[k]);
                    mn = s < mn ? s : mn;
                }
            const u64 kmin = block_min_u64<BLOCK>(mn, s_red);
            if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
            __syncthreads();
            for (i32 k = threadIdx.x; k < ne; k += BLOCK) {
                if (ld_coherent(&lst[k]) == 1 && (u64)ld_coherent((const u64 *)&lsup[k]) == kmin) {
                    const u32 p = atomicAdd(&s_cnt[0], 1u);
                    st_coherent(&lbatch[p], k);
                    st_coherent(&lst[k], (unsigned char)2);
                    a.theta[a.es[base + k]] = kmin;
                }
            }
            __syncthreads();
            const i32 nb = (i32)s_cnt[0];
            if (a.levels && threadIdx.x == 0) atomicAdd(&a.levels[pid], 1u);
            // links of the batch: twin updates and dropped-pair counts
            for (i32 cb = 0; cb < nb; cb += BLOCK) {
                const i32 j = cb + threadIdx.x;
                i32 pl = 0;
                i64 moff = 0;
                i32 own = -1;
                if (j < nb) {
                    const i32 k = ld_coherent(&lbatch[j]);
                    own = a.es[base + k];
                    moff = a.loff[base + k];
                    pl = (i32)(a.loff[base + k + 1] - moff);
                }
                i32 tot;
                const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                s_pre[threadIdx.x] = incl;
                s_moff[threadIdx.x] = moff;
                s_own[threadIdx.x] = own;
                __syncthreads();
                for (i32 q = threadIdx.x; q < tot; q += BLOCK) {
                    int lo = 0, hi = BLOCK - 1;
                    while (lo < hi) {
                        const int md = (lo + hi) >> 1;
                        if (s_pre[md] > q) hi = md; else lo = md + 1;
                    }
                    const i64 li = s_moff[lo] + (q - (lo ? s_pre[lo - 1] : 0));
                    const i32 e = s_own[lo];
                    const i32 et = a.ltwin[li];
                    const u32 t = a.linst[li];
                    ++work;
                    unsigned char ts = 3;  // twin in a higher partition
                    i32 tk = -1;
                    if (a.part[et] == pid) {
                        tk = a.eloc[et];
                        ts = ld_coherent(&lst[tk]);
                    }
                    if (ts == 0) continue;               // pair dropped at a lower level
                    if (ts == 2 && et > e) continue;     // the larger twin acts
                    if (ts == 1) {
                        const u64 kb = ld_coherent(&a.ik[t]);
                        if (kb > 1) atomicAdd((unsigned long long *)&lsup[tk], (unsigned long long)(0ull - (kb - 1)));
                    }
                    if (atomicAdd(&a.icount[t], 1u) == 0) {
                        const u32 p = atomicAdd(&s_cnt[1], 1u);
                        st_coherent(&ltouch[p], t);
                    }
                }
                __syncthreads();
            }
            // touched instances: every surviving pair's partition edges lose count
            const i32 nt = (i32)s_cnt[1];
            for (i32 cb = 0; cb < nt; cb += BLOCK) {
                const i32 j = cb + threadIdx.x;
                i32 pl = 0;
                i64 moff = 0;
                i32 own = -1;
                if (j < nt) {
                    own = (i32)ld_coherent(&ltouch[j]);
                    moff = a.ipstart[own];
                    pl = (i32)ld_coherent(&a.iplen[own]);
                }
                i32 tot;
                const i32 incl = block_incl_scan_i32<BLOCK>(pl, s_wave, tot);
                s_pre[threadIdx.x] = incl;
                s_moff[threadIdx.x] = moff;
                s_own[threadIdx.x] = own;
                __syncthreads();
                for (i32 q = threadIdx.x; q < tot; q += BLOCK) {
                    int lo = 0, hi = BLOCK - 1;
                    while (lo < hi) {
                        const int md = (lo + hi) >> 1;
                        if (s_pre[md] > q) hi = md; else lo = md + 1;
                    }
                    const i64 pq = s_moff[lo] + (q - (lo ? s_pre[lo - 1] : 0));
                    const u32 t = (u32)s_own[lo];
                    const i32 e1 = ld_coherent(&a.fpair[2 * pq]);
                    if (e1 < 0) continue;  // dropped earlier
                    const i32 e2 = ld_coherent(&a.fpair[2 * pq + 1]);
                    ++work;
                    const bool in1 = a.part[e1] == pid, in2 = a.part[e2] == pid;
                    const i32 k1 = in1 ? a.eloc[e1] : -1, k2 = in2 ? a.eloc[e2] : -1;
                    const unsigned char s1 = in1 ? ld_coherent(&lst[k1]) : (unsigned char)1;
                    const unsigned char s2 = in2 ? ld_coherent(&lst[k2]) : (unsigned char)1;
                    if (s1 != 1 || s2 != 1) {
                        st_coherent(&a.fpair[2 * pq], -1);  // drop the pair
                        continue;
                    }
                    const u64 cnt = ld_coherent(&a.icount[t]);
                    if (in1) atomicAdd((unsigned long long *)&lsup[k1], (unsigned long long)(0ull - cnt));
                    if (in2) atomicAdd((unsigned long long *)&lsup[k2], (unsigned long long)(0ull - cnt));
                }
                __syncthreads();
            }
            for (i32 j = threadIdx.x; j < nt; j += BLOCK) {
                const u32 t = ld_coherent(&ltouch[j]);
                const u32 cnt = atomicExch(&a.icount[t], 0u);
                atomicSub(&a.ik[t], cnt);
            }
            // clamp at the level (the clamps of one level commute) and retire
            // the batch
            for (i32 k = threadIdx.x; k < ne; k += BLOCK) {
                const unsigned char s = ld_coherent(&lst[k]);
                if (s == 2) {
                    st_coherent(&lst[k], (unsigned char)0);
                } else if (s == 1) {
                    const i64 v = ld_coherent(&lsup[k]);
                    if (v < (i64)kmin) st_coherent(&lsup[k], (i64)kmin);
                }
            }
            remaining -= nb;
            __syncthreads();
        }
    }
    Tally tl;
    tl.wedges = work;
    tl.flush(a.kc, a.work);
}

// ------------------------------------------------------------------ large partitions
//
// A partition whose work would keep one workgroup busy for long is peeled
// level by level with device-wide kernels instead (the level-batch rule and
// the updates are those of k_wing_fd): every level is one minimum reduction,
// one batch selection, one pass over the batch's links, one over the touched
// instances' pairs, the bloom-number update and the clamp.  Levels are
// issued in groups without waiting; levels after the last find nothing to do.

// All wide partitions advance together: one step peels the current minimum
// level of every wide partition that still has edges, so the number of steps
// is the largest level count among them, not the sum.  State is indexed by
// position in the partition-grouped edge order (es), so an edge e of
// partition p sits at epoff[p] + eloc[e].  Scans over a partition's edges use
// a 2-D grid: blockIdx.y is the wide partition, blockIdx.x strides over its
// edges.

struct WideCtl {
    u32 nb, ntouch;
    u64 alive;  // edges of wide partitions not yet peeled
    u64 steps;
};

constexpr u64 WFD_BIG_WORK = u64(1) << 24;  // estimated work above which a partition goes device-wide
constexpr int WFD_BIG_GROUP = 8;            // steps issued per host check

struct WideArgs {
    const i32 *wpid;    // wide partition -> partition id
    const i64 *epoff;
    const i32 *es;
    const i32 *part;
    const i32 *eloc;
    const i32 *widx;    // partition id -> wide index or -1
    i64 *lsup;          // [m] by position
    unsigned char *lst; // [m] by position: 1 alive, 2 batch, 0 peeled
    u64 *kmin;          // [nw] current level
    u32 *nbw;           // [nw] edges peeled this step
    u64 *remaining;     // [nw]
    u64 *levels;        // [nw]
    i32 *batch;         // positions peeled this step
    u32 *touch;         // instances touched this step
    WideCtl *ctl;
    const u64 *init;
    u64 *theta;
    i32 nw;
};

__global__ void wm_init(WideArgs a) {
    const i32 w = blockIdx.y;
    const i32 pid = a.wpid[w];
    const i64 b = a.epoff[pid], e = a.epoff[pid + 1];
    for (i64 q = b + blockIdx.x * (i64)blockDim.x + threadIdx.x; q < e; q += (i64)gridDim.x * blockDim.x) {
        a.lsup[q] = (i64)a.init[a.es[q]];
        a.lst[q] = 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.kmin[w] = ~0ull;
        a.nbw[w] = 0;
        a.remaining[w] = (u64)(e - b);
        a.levels[w] = 0;
        atomicAdd((unsigned long long *)&a.ctl->alive, (unsigned long long)(e - b));
    }
}

__global__ __launch_bounds__(256) void wm_min(WideArgs a) {
    __shared__ u64 s_red[256 / WAVE];
    const i32 w = blockIdx.y;
    if (a.remaining[w] == 0) return;  // block-uniform
    const i32 pid = a.wpid[w];
    const i64 b = a.epoff[pid], e = a.epoff[pid + 1];
    u64 mn = ~0ull;
    for (i64 q = b + blockIdx.x * (i64)blockDim.x + threadIdx.x; q < e; q += (i64)gridDim.x * blockDim.x)
        if (a.lst[q] == 1) {
            const u64 v = (u64)a.lsup[q];
            mn = v < mn ? v : mn;
        }
    mn = block_min_u64<256>(mn, s_red);
    if (threadIdx.x == 0 && mn != ~0ull) atomicMin((unsigned long long *)&a.kmin[w], (unsigned long long)mn);
}

__global__ void wm_batch(WideArgs a) {
    const i32 w = blockIdx.y;
    if (a.remaining[w] == 0) return;
    const i32 pid = a.wpid[w];
    const i64 b = a.epoff[pid], e = a.epoff[pid + 1];
    const u64 kmin = a.kmin[w];
    u32 cnt = 0;
    for (i64 q = b + blockIdx.x * (i64)blockDim.x + threadIdx.x; q < e; q += (i64)gridDim.x * blockDim.x) {
        if (a.lst[q] == 1 && (u64)a.lsup[q] == kmin) {
            const u32 p = atomicAdd(&a.ctl->nb, 1u);
            a.batch[p] = (i32)q;
            a.lst[q] = 2;
            a.theta[a.es[q]] = kmin;
            ++cnt;
        }
    }
    if (cnt) atomicAdd(&a.nbw[w], cnt);
}

// one wave per batch edge: twin updates (Algorithm 6 reading: k_B - 1) and
// the first touch of every instance
__global__ void wm_links(const WFdArgs f, WideArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 nb = a.ctl->nb;
    u64 work = 0;
    for (i64 j = wave; j < nb; j += nwaves) {
        const i64 q = a.batch[j];
        const i32 e = a.es[q];
        const i32 pid = a.part[e];
        const i64 pbase = a.epoff[pid];
        for (i64 li = f.loff[q] + lane; li < f.loff[q + 1]; li += WAVE) {
            const i32 et = f.ltwin[li];
            const u32 t = f.linst[li];
            ++work;
            unsigned char ts = 3;
            i64 tq = -1;
            if (a.part[et] == pid) {
                tq = pbase + a.eloc[et];
                ts = a.lst[tq];
            }
            if (ts == 0) continue;
            if (ts == 2 && et > e) continue;
            if (ts == 1) {
                const u64 kb = f.ik[t];
                if (kb > 1) atomicAdd((unsigned long long *)&a.lsup[tq], (unsigned long long)(0ull - (kb - 1)));
            }
            if (atomicAdd(&f.icount[t], 1u) == 0) {
                const u32 p = atomicAdd(&a.ctl->ntouch, 1u);
                a.touch[p] = t;
            }
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) work += __shfl_down(work, d, WAVE);
    if (lane == 0 && work) atomicAdd((unsigned long long *)f.work, (unsigned long long)work);
}

// one wave per touched instance: surviving pairs lose the instance's count
__global__ void wm_inst(const WFdArgs f, WideArgs a, const i32 *ipart) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 nt = a.ctl->ntouch;
    u64 work = 0;
    for (i64 j = wave; j < nt; j += nwaves) {
        const u32 t = a.touch[j];
        const i32 pid = ipart[t];
        const i64 pbase = a.epoff[pid];
        const u64 cnt = f.icount[t];
        const i64 p0 = f.ipstart[t];
        const i64 p1 = p0 + f.iplen[t];
        for (i64 pq = p0 + lane; pq < p1; pq += WAVE) {
            const i32 e1 = f.fpair[2 * pq];
            if (e1 < 0) continue;
            const i32 e2 = f.fpair[2 * pq + 1];
            ++work;
            const bool in1 = a.part[e1] == pid, in2 = a.part[e2] == pid;
            const i64 q1 = in1 ? pbase + a.eloc[e1] : -1, q2 = in2 ? pbase + a.eloc[e2] : -1;
            const unsigned char s1 = in1 ? a.lst[q1] : (unsigned char)1;
            const unsigned char s2 = in2 ? a.lst[q2] : (unsigned char)1;
            if (s1 != 1 || s2 != 1) {
                f.fpair[2 * pq] = -1;
                continue;
            }
            if (in1) atomicAdd((unsigned long long *)&a.lsup[q1], (unsigned long long)(0ull - cnt));
            if (in2) atomicAdd((unsigned long long *)&a.lsup[q2], (unsigned long long)(0ull - cnt));
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) work += __shfl_down(work, d, WAVE);
    if (lane == 0 && work) atomicAdd((unsigned long long *)f.work, (unsigned long long)work);
}

__global__ void wm_reset(const WFdArgs f, WideArgs a) {
    const u32 nt = a.ctl->ntouch;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < nt; j += gridDim.x * blockDim.x) {
        const u32 t = a.touch[j];
        const u32 cnt = f.icount[t];
        f.icount[t] = 0;
        f.ik[t] -= cnt;
    }
}

__global__ void wm_clamp(WideArgs a) {
    const i32 w = blockIdx.y;
    if (a.remaining[w] == 0) return;
    const u64 kmin = a.kmin[w];
    if (kmin == ~0ull) return;
    const i32 pid = a.wpid[w];
    const i64 b = a.epoff[pid], e = a.epoff[pid + 1];
    for (i64 q = b + blockIdx.x * (i64)blockDim.x + threadIdx.x; q < e; q += (i64)gridDim.x * blockDim.x) {
        const unsigned char st = a.lst[q];
        if (st == 2) {
            a.lst[q] = 0;
        } else if (st == 1 && a.lsup[q] < (i64)kmin) {
            a.lsup[q] = (i64)kmin;
        }
    }
}

__global__ void wm_next(WideArgs a) {
    for (i32 w = blockIdx.x * blockDim.x + threadIdx.x; w < a.nw; w += gridDim.x * blockDim.x) {
        const u32 nb = a.nbw[w];
        if (nb) {
            a.remaining[w] -= nb;
            a.levels[w] += 1;
            atomicAdd((unsigned long long *)&a.ctl->alive, (unsigned long long)(0ull - (u64)nb));
        }
        a.nbw[w] = 0;
        a.kmin[w] = ~0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->nb = 0;
        a.ctl->ntouch = 0;
        a.ctl->steps += 1;
    }
}

// ------------------------------------------------------------------ host

static double wnow_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Default P (Section 6.1 settings) and the work-efficiency clamp of
// Section 4.2 (wing: P at most the support total over m).
static int wing_partitions(const pbng_opts &o, u64 sup_total, i64 m) {
    if (o.P > 0) return o.P;
    int P = m >= 100000000 ? 1000 : 400;
    double cap = m > 0 ? std::floor((double)sup_total / (double)m) : 1.0;
    if (cap < 1) cap = 1;
    if (P > cap) P = (int)cap;
    return std::max(P, 1);
}

void wing_decompose(Ctx &c, const DevGraph &G, const pbng_opts &o, u64 *theta) {
    hipStream_t s = c.stream;
    const i64 m = G.m;
    if (m == 0) return;
    const bool dynamic = !(o.flags & PBNG_F_NO_DYNAMIC);
    // PBNG--: per-edge bloom walks instead of bloom-aggregated batches
    const bool unbatched = (o.flags & PBNG_F_NO_BATCH) != 0;
    const double t0 = wnow_ms();

    // ---- per-edge counting and BE-Index
    u64 *sup = c.alloc<u64>(m);
    BEIndex I;
    build_be_index(c, G, I, sup);
    PBNG_HIP(hipStreamSynchronize(s));
    const double t1 = wnow_ms();
    c.stats.ms_count = t1 - t0;
    const i64 nbl = I.nblooms, npr = I.npairs;

    // CD works on a copy of the pair lists (it drops pairs); FD partitions the
    // original index
    i32 *cedge = c.alloc<i32>(2 * npr);
    if (npr) PBNG_HIP(hipMemcpyAsync(cedge, I.bedge, sizeof(i32) * 2 * npr, hipMemcpyDeviceToDevice, s));
    u32 *bk = c.alloc<u32>(nbl);
    if (nbl) PBNG_HIP(hipMemcpyAsync(bk, I.bk, sizeof(u32) * nbl, hipMemcpyDeviceToDevice, s));
    u32 *blen = c.alloc<u32>(nbl);
    u32 *bcount = c.alloc<u32>(nbl);
    i32 *touched = c.alloc<i32>(nbl);
    if (nbl) {
        hipLaunchKernelGGL(w_blen_init, dim3(grid_1d(nbl)), dim3(256), 0, s, (const i64 *)I.boff, nbl, blen);
        PBNG_HIP(hipMemsetAsync(bcount, 0, sizeof(u32) * nbl, s));
        PBNG_LAUNCH_CHECK();
    }
    unsigned char *st = c.alloc<unsigned char>(m);
    i32 *part = c.alloc<i32>(m);
    u64 *init = c.alloc<u64>(m);
    i32 *F = c.alloc<i32>(m);
    i32 *F2 = c.alloc<i32>(m);
    WingCtl *ctl = c.alloc<WingCtl>(1);
    u64 *rmm = c.alloc<u64>(2);
    PBNG_HIP(hipMemsetAsync(st, 0, m, s));
    PBNG_HIP(hipMemsetAsync(ctl, 0, sizeof(WingCtl), s));
    {
        double one = 1.0;
        PBNG_HIP(hipMemcpyAsync(&ctl->scale, &one, sizeof(double), hipMemcpyHostToDevice, s));
    }
    const u64 sup_total = reduce_sum_u64(c, sup, m);
    const int P = wing_partitions(o, sup_total, m);
    c.stats.P_used = P;
    const int gm = grid_1d(m);

    // ---- coarse-grained phase
    // Rounds are either driven from the host (one synchronisation per round
    // to read the active-set size) or captured once into a HIP graph of
    // W_GRAPH_K rounds with fixed grids that is replayed until the active set
    // is empty (one synchronisation per replay).  Rounds past the end of a
    // partition find an empty active set and do nothing.
    const bool host_rounds = (o.flags & PBNG_F_HOST_ROUNDS) != 0;
    const int gfix = c.num_cu * 8;
    auto links = [&](hipStream_t rs, dim3 grid, i32 *Fa, i32 *Fb) {
        if (unbatched)
            hipLaunchKernelGGL(w_links_each, grid, dim3(256), 0, rs, (const i32 *)Fa, (const u32 *)&ctl->nF,
                               (const i64 *)I.eoff, (const i32 *)I.ebloom, (const i32 *)I.etwin, (const unsigned char *)st,
                               (const u32 *)bk, bcount, touched, (const i64 *)I.boff, (const u32 *)blen,
                               (const i32 *)cedge, sup, ctl, Fb, c.kctr + PBNG_K_WING_CD);
        else
            hipLaunchKernelGGL(w_links, grid, dim3(256), 0, rs, (const i32 *)Fa, (const u32 *)&ctl->nF, (const i64 *)I.eoff,
                               (const i32 *)I.ebloom, (const i32 *)I.etwin, (const unsigned char *)st, (const u32 *)bk,
                               bcount, touched, sup, ctl, Fb, c.kctr + PBNG_K_WING_CD);
    };
    auto round_fixed = [&](hipStream_t rs, i32 *Fa, i32 *Fb) {
        links(rs, dim3(gfix), Fa, Fb);
        hipLaunchKernelGGL(w_blooms, dim3(gfix), dim3(256), 0, rs, (const i32 *)touched, (const u32 *)&ctl->ntouch,
                           (const i64 *)I.boff, blen, bk, bcount, cedge, (const unsigned char *)st, sup, ctl, Fb,
                           dynamic ? 1 : 0, unbatched ? 0 : 1, c.kctr + PBNG_K_WING_CD);
        hipLaunchKernelGGL(w_retire, dim3(c.num_cu * 2), dim3(256), 0, rs, (const i32 *)Fa, (const u32 *)&ctl->nF, st,
                           (const u64 *)init, ctl);
        hipLaunchKernelGGL(w_activate, dim3(c.num_cu * 2), dim3(256), 0, rs, (const i32 *)Fb, (const u32 *)&ctl->nF2, st,
                           part, (const WingCtl *)ctl);
        hipLaunchKernelGGL(w_next_round, dim3(1), dim3(1), 0, rs, ctl);
    };
    GraphExec rounds_exec;
    if (!host_rounds) {
        hipStream_t cs = c.capture_stream();
        PBNG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        i32 *Fa = F, *Fb = F2;
        for (int r = 0; r < W_GRAPH_K; ++r) {
            round_fixed(cs, Fa, Fb);
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
    hipLaunchKernelGGL(w_alive_init, dim3(1), dim3(1), 0, s, ctl, m);
    i64 n_alive = m;
    int pid = 0;
    u64 rho = 0;
    while (n_alive > 0) {
        const bool last = (P - pid) <= 1;
        if (!last) {
            if (o.bound_rule == PBNG_BOUND_RANDOM) {
                u64 init2[2] = {~0ull, 0};
                PBNG_HIP(hipMemcpyAsync(rmm, init2, sizeof(init2), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(w_minmax, dim3(gm), dim3(256), 0, s, (const u64 *)sup, (const unsigned char *)st, m, rmm,
                                   rmm + 1);
                hipLaunchKernelGGL(w_random_pick, dim3(1), dim3(1), 0, s, ctl, (const u64 *)rmm, (const u64 *)(rmm + 1),
                                   (u64)o.seed, pid);
                PBNG_LAUNCH_CHECK();
            } else {
                // work estimate of an edge: its support (Algorithm 4, find_range)
                weighted_select(c, sup, sup, st, WS_ALIVE, m, nullptr, &ctl->scale, P - pid, &ctl->s, &ctl->est_init);
            }
        }
        hipLaunchKernelGGL(w_set_bound, dim3(1), dim3(1), 0, s, ctl, last ? 1 : 0, (i32)pid);
        hipLaunchKernelGGL(w_frontier, dim3(gm), dim3(256), 0, s, st, (const u64 *)sup, init, part, m, ctl, pid, F);
        PBNG_LAUNCH_CHECK();
        if (!host_rounds) {
            for (;;) {
                WingCtl h;
                PBNG_HIP(hipMemcpyAsync(&h, ctl, sizeof(WingCtl), hipMemcpyDeviceToHost, s));
                PBNG_HIP(hipStreamSynchronize(s));
                n_alive = h.alive;
                if (h.nF == 0) break;
                if ((i64)h.nF == h.alive) {
                    // everything left is active: retire it without updates
                    hipLaunchKernelGGL(w_retire, dim3(grid_1d(h.nF)), dim3(256), 0, s, (const i32 *)F,
                                       (const u32 *)&ctl->nF, st, (const u64 *)init, ctl);
                    PBNG_LAUNCH_CHECK();
                    ++rho;
                    n_alive = 0;
                    break;
                }
                c.kbegin(PBNG_K_WING_CD);
                PBNG_HIP(hipGraphLaunch(rounds_exec.e, s));
                c.kend(PBNG_K_WING_CD);
            }
        } else {
            u32 nF = read_scalar<u32>(c, &ctl->nF);
            while (nF > 0) {
                ++rho;
                const int gw = grid_1d((i64)nF * WAVE);
                if ((i64)nF == n_alive) {
                    hipLaunchKernelGGL(w_retire, dim3(grid_1d(nF)), dim3(256), 0, s, (const i32 *)F, (const u32 *)&ctl->nF, st,
                                       (const u64 *)init, ctl);
                    PBNG_LAUNCH_CHECK();
                    n_alive = 0;
                    break;
                }
                c.kbegin(PBNG_K_WING_CD);
                links(s, dim3(gw), F, F2);
                PBNG_LAUNCH_CHECK();
                hipLaunchKernelGGL(w_blooms, dim3(grid_1d((i64)std::min<i64>(nbl, (i64)nF * 64) * WAVE)), dim3(256), 0, s,
                                   (const i32 *)touched, (const u32 *)&ctl->ntouch, (const i64 *)I.boff, blen, bk, bcount,
                                   cedge, (const unsigned char *)st, sup, ctl, F2, dynamic ? 1 : 0, unbatched ? 0 : 1,
                                   c.kctr + PBNG_K_WING_CD);
                c.kend(PBNG_K_WING_CD);
                PBNG_LAUNCH_CHECK();
                hipLaunchKernelGGL(w_retire, dim3(grid_1d(nF)), dim3(256), 0, s, (const i32 *)F, (const u32 *)&ctl->nF, st,
                                   (const u64 *)init, ctl);
                hipLaunchKernelGGL(w_activate, dim3(gm), dim3(256), 0, s, (const i32 *)F2, (const u32 *)&ctl->nF2, st, part,
                                   (const WingCtl *)ctl);
                hipLaunchKernelGGL(w_next_round, dim3(1), dim3(1), 0, s, ctl);
                PBNG_LAUNCH_CHECK();
                n_alive -= nF;
                std::swap(F, F2);
                nF = read_scalar<u32>(c, &ctl->nF);
            }
        }
        hipLaunchKernelGGL(w_scale, dim3(1), dim3(1), 0, s, ctl);
        PBNG_LAUNCH_CHECK();
        ++pid;
    }
    if (!host_rounds) rho += read_scalar<u64>(c, &ctl->rounds);
    const i32 np = pid;
    c.stats.rho = rho;
    c.stats.partitions = np;
    c.stats.updates = read_scalar<u64>(c, &ctl->updates);
    c.stats.links = read_scalar<u64>(c, &ctl->links);
    const double t2 = wnow_ms();
    c.stats.ms_cd = t2 - t1;

    // ---- fine-grained preparation: partition_BE_Index
    // edges grouped by partition
    u64 *ek = c.alloc<u64>(m);
    i32 *ev = c.alloc<i32>(m);
    u32 *pcount = c.alloc<u32>(np);
    PBNG_HIP(hipMemsetAsync(pcount, 0, sizeof(u32) * np, s));
    hipLaunchKernelGGL(w_part_keys, dim3(gm), dim3(256), 0, s, (const i32 *)part, m, ek, ev);
    hist_add_u32(c, part, m, np, pcount);
    PBNG_LAUNCH_CHECK();
    u64 *eks;
    i32 *es;
    radix_sort_u64(c, ek, ev, m, bits_for((u64)np), &eks, &es);
    i64 *pc64 = c.alloc<i64>(np);
    i64 *epoff = c.alloc<i64>(np + 1);
    hipLaunchKernelGGL(w_u32_to_i64, dim3(grid_1d(np)), dim3(256), 0, s, (const u32 *)pcount, (i64)np, pc64);
    exclusive_scan<i64>(c, pc64, epoff, np);
    i32 *eloc = c.alloc<i32>(m);
    hipLaunchKernelGGL(w_loc, dim3(gm), dim3(256), 0, s, (const i32 *)es, (const i32 *)part, (const i64 *)epoff, m, eloc);
    PBNG_LAUNCH_CHECK();

    // pairs: bloom numbers per partition instance, then (partition, bloom) order
    u32 *pk = c.alloc<u32>(npr);
    i32 *fpair = c.alloc<i32>(2 * npr);
    u32 *isstart = c.alloc<u32>(npr);
    u32 *iexcl = c.alloc<u32>(npr + 1);
    u32 *pinst = c.alloc<u32>(npr);
    i64 ninst = 0;
    i64 *ipstart = nullptr;
    u32 *ik = nullptr, *iplen = nullptr, *icount = nullptr;
    i32 *ipart = nullptr;
    if (npr) {
        u64 *k1 = c.alloc<u64>(npr);
        i32 *v1 = c.alloc<i32>(npr);
        hipLaunchKernelGGL(w_pair_keys_bp, dim3(grid_1d(npr)), dim3(256), 0, s, (const i32 *)I.bedge, (const i32 *)I.pbloom,
                           (const i32 *)part, npr, np, k1, v1);
        PBNG_LAUNCH_CHECK();
        u64 *sk1;
        i32 *sv1;
        radix_sort_u64(c, k1, v1, npr, bits_for((u64)nbl * (u64)np), &sk1, &sv1);
        hipLaunchKernelGGL(w_pair_k, dim3(grid_1d(npr)), dim3(256), 0, s, (const u64 *)sk1, (const i32 *)sv1,
                           (const i64 *)I.boff, (const i32 *)I.pbloom, npr, pk);
        PBNG_LAUNCH_CHECK();
        u64 *k2 = c.alloc<u64>(npr);
        i32 *v2 = c.alloc<i32>(npr);
        hipLaunchKernelGGL(w_pair_keys_pb, dim3(grid_1d(npr)), dim3(256), 0, s, (const i32 *)I.bedge, (const i32 *)I.pbloom,
                           (const i32 *)part, npr, nbl, k2, v2);
        PBNG_LAUNCH_CHECK();
        u64 *sk2;
        i32 *sv2;
        radix_sort_u64(c, k2, v2, npr, bits_for((u64)np * (u64)nbl), &sk2, &sv2);
        hipLaunchKernelGGL(w_fd_pairs, dim3(grid_1d(npr)), dim3(256), 0, s, (const u64 *)sk2, (const i32 *)sv2,
                           (const i32 *)I.bedge, npr, fpair, isstart);
        PBNG_LAUNCH_CHECK();
        exclusive_scan<u32>(c, isstart, iexcl, npr);
        ninst = read_scalar<u32>(c, iexcl + npr);
        ipstart = c.alloc<i64>(ninst);
        ik = c.alloc<u32>(ninst);
        iplen = c.alloc<u32>(ninst);
        icount = c.alloc<u32>(ninst);
        ipart = c.alloc<i32>(ninst);
        hipLaunchKernelGGL(w_fd_instances, dim3(grid_1d(npr)), dim3(256), 0, s, (const u64 *)sk2, (const i32 *)sv2,
                           (const u32 *)isstart, (const u32 *)iexcl, npr, nbl, (const u32 *)pk, ipstart, ik, ipart, pinst);
        hipLaunchKernelGGL(w_fd_instance_len, dim3(grid_1d(ninst)), dim3(256), 0, s, (const i64 *)ipstart, ninst, npr, iplen);
        PBNG_HIP(hipMemsetAsync(icount, 0, sizeof(u32) * (ninst ? ninst : 1), s));
        PBNG_LAUNCH_CHECK();
    }
    // links of the partition edges, in es order
    u32 *lcnt = c.alloc<u32>(m);
    i64 *lcnt64 = c.alloc<i64>(m);
    i64 *loff = c.alloc<i64>(m + 1);
    PBNG_HIP(hipMemsetAsync(lcnt, 0, sizeof(u32) * m, s));
    if (npr) {
        hipLaunchKernelGGL(w_fd_link_count, dim3(grid_1d(npr)), dim3(256), 0, s, (const i32 *)fpair, (const u32 *)pinst,
                           (const i32 *)ipart, (const i32 *)part, (const i64 *)epoff, (const i32 *)eloc, npr, lcnt);
        PBNG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(w_u32_to_i64, dim3(gm), dim3(256), 0, s, (const u32 *)lcnt, m, lcnt64);
    exclusive_scan<i64>(c, lcnt64, loff, m);
    const i64 nlinks = read_scalar<i64>(c, loff + m);
    u32 *linst = c.alloc<u32>(nlinks);
    i32 *ltwin = c.alloc<i32>(nlinks);
    if (npr) {
        i64 *lcur = c.alloc<i64>(m);
        PBNG_HIP(hipMemcpyAsync(lcur, loff, sizeof(i64) * m, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(w_fd_link_fill, dim3(grid_1d(npr)), dim3(256), 0, s, (const i32 *)fpair, (const u32 *)pinst,
                           (const i32 *)ipart, (const i32 *)part, (const i64 *)epoff, (const i32 *)eloc, npr, lcur, linst,
                           ltwin);
        PBNG_LAUNCH_CHECK();
    }
    // LPT order by the partitions' total initial support
    u64 *work = c.alloc<u64>(np);
    u64 *wm = c.alloc<u64>(4);
    PBNG_HIP(hipMemsetAsync(work, 0, sizeof(u64) * np, s));
    PBNG_HIP(hipMemsetAsync(wm, 0, 4 * sizeof(u64), s));
    hist_add_u64(c, part, init, m, np, work);
    hipLaunchKernelGGL(w_max_u64, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)work, (i64)np, wm, wm + 1);
    hipLaunchKernelGGL(w_max_u64, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)pc64, (i64)np, wm + 2, (u64 *)nullptr);
    PBNG_LAUNCH_CHECK();
    const u64 maxw = read_scalar<u64>(c, wm);
    c.stats.fd_work_max = maxw;
    c.stats.fd_work_sum = read_scalar<u64>(c, wm + 1);
    const i64 maxne = std::max<i64>((i64)read_scalar<u64>(c, wm + 2), 1);
    i64 maxinst = 1;
    if (ninst) {
        u32 *icnt = c.alloc<u32>(np);
        i64 *icnt64 = c.alloc<i64>(np);
        PBNG_HIP(hipMemsetAsync(icnt, 0, sizeof(u32) * np, s));
        hist_add_u32(c, ipart, ninst, np, icnt);
        hipLaunchKernelGGL(w_u32_to_i64, dim3(grid_1d(np)), dim3(256), 0, s, (const u32 *)icnt, (i64)np, icnt64);
        PBNG_HIP(hipMemsetAsync(wm + 3, 0, sizeof(u64), s));
        hipLaunchKernelGGL(w_max_u64, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)icnt64, (i64)np, wm + 3, (u64 *)nullptr);
        PBNG_LAUNCH_CHECK();
        maxinst = std::max<i64>((i64)read_scalar<u64>(c, wm + 3), 1);
    }
    u64 *lk = c.alloc<u64>(np);
    i32 *lv = c.alloc<i32>(np);
    hipLaunchKernelGGL(w_lpt_keys, dim3(grid_1d(np)), dim3(256), 0, s, (const u64 *)work, np, maxw, lk, lv);
    PBNG_LAUNCH_CHECK();
    u64 *lks;
    i32 *queue;
    radix_sort_u64(c, lk, lv, np, bits_for(maxw), &lks, &queue);
    PBNG_HIP(hipStreamSynchronize(s));
    const double t3 = wnow_ms();
    c.stats.ms_fd_prep = t3 - t2;

    // ---- fine-grained phase
    // partitions in LPT order; the largest (work above WFD_BIG_WORK) are
    // peeled device-wide on the context stream while the persistent kernel
    // takes the rest from the queue on a second stream
    std::vector<i32> q_h(np);
    std::vector<u64> w_h(np);
    std::vector<i64> eo_h(np + 1);
    PBNG_HIP(hipMemcpyAsync(q_h.data(), queue, sizeof(i32) * np, hipMemcpyDeviceToHost, s));
    PBNG_HIP(hipMemcpyAsync(w_h.data(), work, sizeof(u64) * np, hipMemcpyDeviceToHost, s));
    PBNG_HIP(hipMemcpyAsync(eo_h.data(), epoff, sizeof(i64) * (np + 1), hipMemcpyDeviceToHost, s));
    PBNG_HIP(hipStreamSynchronize(s));
    const bool big_off = o.wide_work < 0;
    const u64 big_work = o.wide_work > 0 ? (u64)o.wide_work : WFD_BIG_WORK;
    u32 nbig = 0;
    i64 big_ne = 1;  // edges of the largest wide partition
    while (!big_off && (i32)nbig < np && w_h[q_h[nbig]] >= big_work) {
        big_ne = std::max<i64>(big_ne, eo_h[q_h[nbig] + 1] - eo_h[q_h[nbig]]);
        ++nbig;
    }
    const i32 nsmall = np - (i32)nbig;
    const int fdblocks = (int)std::max<i64>(1, std::min<i64>(nsmall, (i64)c.num_cu * 2));
    WFdArgs fa{};
    fa.es = es;
    fa.epoff = epoff;
    fa.eloc = eloc;
    fa.part = part;
    fa.loff = loff;
    fa.linst = linst;
    fa.ltwin = ltwin;
    fa.ipstart = ipstart;
    fa.iplen = iplen;
    fa.ik = ik;
    fa.icount = icount;
    fa.fpair = fpair;
    fa.queue = queue;
    fa.np = np;
    fa.head = c.alloc<u32>(1);
    PBNG_HIP(hipMemcpyAsync(fa.head, &nbig, sizeof(u32), hipMemcpyHostToDevice, s));
    fa.init = init;
    fa.theta = theta;
    fa.maxne = maxne;
    fa.lsup = c.alloc<i64>((i64)fdblocks * maxne);
    fa.lst = c.alloc<unsigned char>((i64)fdblocks * maxne);
    fa.lbatch = c.alloc<i32>((i64)fdblocks * maxne);
    fa.tstride = maxinst;
    fa.ltouch = c.alloc<u32>((i64)fdblocks * maxinst);
    fa.work = c.alloc<u64>(1);
    fa.kc = c.kctr + PBNG_K_FD;
    PBNG_HIP(hipMemsetAsync(fa.work, 0, sizeof(u64), s));
    const bool trace = getenv("PBNG_TRACE") != nullptr;
    if (trace) {
        fa.levels = c.alloc<u32>(np);
        PBNG_HIP(hipMemsetAsync(fa.levels, 0, sizeof(u32) * np, s));
    }
    // wide-partition state
    WideArgs wa{};
    std::vector<i32> wpid_h(q_h.begin(), q_h.begin() + nbig);
    std::vector<i32> widx_h(np, -1);
    for (u32 b = 0; b < nbig; ++b) widx_h[q_h[b]] = (i32)b;
    std::vector<u64> big_levels(nbig, 0);
    c.kbegin(PBNG_K_FD);
    StreamJoin join(c);
    if (nsmall > 0) {
        join.fork();
        hipLaunchKernelGGL(k_wing_fd, dim3(fdblocks), dim3(256), 0, join.aux, fa);
        PBNG_LAUNCH_CHECK();
    }
    if (nbig > 0) {
        i32 *wpid = c.alloc<i32>(nbig);
        i32 *widx = c.alloc<i32>(np);
        PBNG_HIP(hipMemcpy(wpid, wpid_h.data(), sizeof(i32) * nbig, hipMemcpyHostToDevice));
        PBNG_HIP(hipMemcpy(widx, widx_h.data(), sizeof(i32) * np, hipMemcpyHostToDevice));
        wa.wpid = wpid;
        wa.epoff = epoff;
        wa.es = es;
        wa.part = part;
        wa.eloc = eloc;
        wa.widx = widx;
        wa.lsup = c.alloc<i64>(m);
        wa.lst = c.alloc<unsigned char>(m);
        wa.kmin = c.alloc<u64>(nbig);
        wa.nbw = c.alloc<u32>(nbig);
        wa.remaining = c.alloc<u64>(nbig);
        wa.levels = c.alloc<u64>(nbig);
        wa.batch = c.alloc<i32>(m);
        wa.touch = c.alloc<u32>(std::max<i64>(ninst, 1));
        wa.ctl = c.alloc<WideCtl>(1);
        wa.init = init;
        wa.theta = theta;
        wa.nw = (i32)nbig;
        PBNG_HIP(hipMemsetAsync(wa.ctl, 0, sizeof(WideCtl), s));
        const dim3 g2((unsigned)std::max<i64>(1, std::min<i64>((big_ne + 1023) / 1024, 64)), nbig);
        const int gb = c.num_cu * 4;
        hipLaunchKernelGGL(wm_init, g2, dim3(256), 0, s, wa);
        PBNG_LAUNCH_CHECK();
        u64 alive = 1;
        // every step retires at least one edge of every unfinished partition
        for (i64 groups = 0; alive > 0; ++groups) {
            if (groups > big_ne / WFD_BIG_GROUP + 2) throw Error(PBNG_E_DEVICE, "wide partitions did not finish");
            for (int l = 0; l < WFD_BIG_GROUP; ++l) {
                hipLaunchKernelGGL(wm_min, g2, dim3(256), 0, s, wa);
                hipLaunchKernelGGL(wm_batch, g2, dim3(256), 0, s, wa);
                hipLaunchKernelGGL(wm_links, dim3(gb), dim3(256), 0, s, fa, wa);
                hipLaunchKernelGGL(wm_inst, dim3(gb), dim3(256), 0, s, fa, wa, (const i32 *)ipart);
                hipLaunchKernelGGL(wm_reset, dim3(gb), dim3(256), 0, s, fa, wa);
                hipLaunchKernelGGL(wm_clamp, g2, dim3(256), 0, s, wa);
                hipLaunchKernelGGL(wm_next, dim3(std::max<i64>(1, (nbig + 255) / 256)), dim3(256), 0, s, wa);
                PBNG_LAUNCH_CHECK();
            }
            WideCtl h;
            PBNG_HIP(hipMemcpyAsync(&h, wa.ctl, sizeof(WideCtl), hipMemcpyDeviceToHost, s));
            PBNG_HIP(hipStreamSynchronize(s));
            alive = h.alive;
        }
        PBNG_HIP(hipMemcpyAsync(big_levels.data(), wa.levels, sizeof(u64) * nbig, hipMemcpyDeviceToHost, s));
    }
    join.join();
    c.kend(PBNG_K_FD);
    c.stats.fd_wide = nbig;
    if (trace) {
        std::vector<u32> lv_h(np);
        PBNG_HIP(hipMemcpyAsync(lv_h.data(), fa.levels, sizeof(u32) * np, hipMemcpyDeviceToHost, s));
        PBNG_HIP(hipStreamSynchronize(s));
        for (u32 b = 0; b < nbig; ++b) lv_h[q_h[b]] = (u32)big_levels[b];
        for (int p = 0; p < np; ++p)
            fprintf(stderr, "[pbng-trace] wing-fd part %d edges %lld levels %u work %llu%s\n", p, (long long)(eo_h[p + 1] - eo_h[p]),
                    lv_h[p], (unsigned long long)w_h[p], w_h[p] >= big_work && !big_off ? " wide" : "");
    }
    c.stats.wedges_fd = read_scalar<u64>(c, fa.work);
    c.stats.ms_fd = wnow_ms() - t3;
    c.stats.wedges = c.stats.wedges_count + c.stats.links + c.stats.wedges_fd;
}

}  // namespace pbng
