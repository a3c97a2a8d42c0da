// k-tips and k-wings from entity numbers (Section 2.2, Definitions 1-2).
//
// The k-tips of a side are the butterfly-connected components of its
// vertices with tip number >= k (with all of the other side): two such
// vertices are joined when they share at least two neighbours.  The k-wings
// are the butterfly-connected components of the edges with wing number >= k:
// for a pair of U vertices u < u' whose common neighbours over those edges
// number c >= 2, every two of the c wedges u - v - u' form a butterfly, so
// all 2c edges are joined.  Both come from one wedge walk per start vertex:
// a workgroup counts c(start, last) for the later vertices `last` in HBM
// counters of its own (with a touched list), then joins.  Joins go to a
// union-find forest whose roots only ever move to smaller ids, so a
// component's root is its smallest member.
#include <algorithm>

#include "dev_common.h"
#include "pbng_internal.h"

namespace pbng {

namespace {

__device__ __forceinline__ i32 uf_root(i32 *p, i32 x) {
    for (;;) {
        const i32 q = __hip_atomic_load(&p[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (q == x) return x;
        x = q;
    }
}

__device__ __forceinline__ void uf_unite(i32 *p, i32 a, i32 b) {
    for (;;) {
        a = uf_root(p, a);
        b = uf_root(p, b);
        if (a == b) return;
        if (a > b) {
            const i32 t = a;
            a = b;
            b = t;
        }
        // link the larger root under the smaller one, unless b stopped being a root
        if (atomicCAS(&p[b], b, a) == b) return;
    }
}

__global__ void h_init(i32 *p, i64 n) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = (i32)i;
}

__global__ void h_label(i32 *p, const u64 *theta, u64 k, i64 n, i32 *comp) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        comp[i] = theta[i] >= k ? uf_root(p, (i32)i) : -1;
}

struct HArgs {
    const i64 *xrow;   // start side rows
    const i32 *xadj;
    const i32 *xeid;   // edge id of each start-side entry (wing)
    const i64 *yrow;   // other side rows
    const i32 *yadj;
    const i32 *yeid;   // edge id of each other-side entry (wing)
    const u64 *theta;  // tip numbers of the start side, or wing numbers per edge
    u64 k;
    i64 nx;
    u32 *cnt;          // [grid][nx] counters per workgroup
    i32 *e0;           // [grid][nx] first edge (u, v) per later vertex (wing)
    i32 *touch;        // [grid][nx]
    u32 *next;
    i32 *p;            // union-find forest
    int wing;
};

constexpr int HB = 256;

// One start per workgroup at a time.  Wedges start - y - last are walked by
// chunks of BLOCK neighbours: each thread takes a neighbour's list length
// (its counted part), a block scan lays them out, and threads take wedges
// by index.  pass 0 counts, pass 1 joins (wing only).
template <class F>
__device__ __forceinline__ void walk(const HArgs &a, i32 x, i32 *s_pre, i64 *s_off, i32 *s_e, i32 *s_wave, F fn) {
    const i64 jb = a.xrow[x], je = a.xrow[x + 1];
    for (i64 cb = jb; cb < je; cb += HB) {
        const i64 j = cb + threadIdx.x;
        i32 len = 0;
        i64 off = 0;
        i32 e = -1;
        if (j < je) {
            const bool in = a.wing ? a.theta[a.xeid[j]] >= a.k : true;
            if (in) {
                const i32 y = a.xadj[j];
                off = a.yrow[y];
                len = (i32)(a.yrow[y + 1] - off);
                e = a.wing ? a.xeid[j] : -1;
            }
        }
        i32 tot;
        const i32 incl = block_incl_scan_i32<HB>(len, s_wave, tot);
        s_pre[threadIdx.x] = incl;
        s_off[threadIdx.x] = off;
        s_e[threadIdx.x] = e;
        __syncthreads();
        for (i32 w = threadIdx.x; w < tot; w += HB) {
            int lo = 0, hi = HB - 1;
            while (lo < hi) {
                const int md = (lo + hi) >> 1;
                if (s_pre[md] > w) hi = md; else lo = md + 1;
            }
            const i64 q = s_off[lo] + (w - (lo ? s_pre[lo - 1] : 0));
            fn(s_e[lo], q);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(HB) void h_pairs(HArgs a) {
    __shared__ i32 s_pre[HB];
    __shared__ i64 s_off[HB];
    __shared__ i32 s_e[HB];
    __shared__ i32 s_wave[HB / WAVE];
    __shared__ u32 s_item, s_nt;
    u32 *cnt = a.cnt + (i64)blockIdx.x * a.nx;
    i32 *e0 = a.wing ? a.e0 + (i64)blockIdx.x * a.nx : nullptr;
    i32 *touch = a.touch + (i64)blockIdx.x * a.nx;
    if (threadIdx.x == 0) s_nt = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.next, 1u);
        __syncthreads();
        const i64 x = s_item;
        if (x >= a.nx) break;
        if (!a.wing && a.theta[x] < a.k) continue;  // workgroup-uniform
        // pass 0: c(x, last) for later vertices `last` in the level set
        walk(a, (i32)x, s_pre, s_off, s_e, s_wave, [&](i32 e, i64 q) {
            const i32 l = a.yadj[q];
            if (l <= x) return;
            if (a.wing ? a.theta[a.yeid[q]] < a.k : a.theta[l] < a.k) return;
            if (atomicAdd(&cnt[l], 1u) == 0u) {
                if (a.wing) e0[l] = e;
                touch[atomicAdd(&s_nt, 1u)] = l;
            }
        });
        __syncthreads();
        const u32 nt = s_nt;
        if (a.wing) {
            // pass 1: every wedge of a pair with c >= 2 joins its two edges
            // and the pair's first edge
            walk(a, (i32)x, s_pre, s_off, s_e, s_wave, [&](i32 e, i64 q) {
                const i32 l = a.yadj[q];
                if (l <= x) return;
                const i32 f = a.yeid[q];
                if (a.theta[f] < a.k) return;
                if (cnt[l] >= 2u) {
                    uf_unite(a.p, e, f);
                    uf_unite(a.p, e, e0[l]);
                }
            });
        }
        for (u32 t = threadIdx.x; t < nt; t += HB) {
            const i32 l = touch[t];
            if (!a.wing && cnt[l] >= 2u) uf_unite(a.p, (i32)x, l);
            cnt[l] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_nt = 0;
    }
}

}  // namespace

void level_components(Ctx &c, const DevGraph &G, int what, const u64 *theta, u64 k, i32 *comp) {
    // what: 0 tip numbers of U, 1 tip numbers of V, 2 wing numbers
    hipStream_t s = c.stream;
    HArgs a{};
    const bool wing = what == 2;
    a.wing = wing ? 1 : 0;
    a.xrow = what == 1 ? G.vrow : G.urow;
    a.xadj = what == 1 ? G.vadj : G.ucol;
    a.yrow = what == 1 ? G.urow : G.vrow;
    a.yadj = what == 1 ? G.ucol : G.vadj;
    a.theta = theta;
    a.k = k;
    a.nx = what == 1 ? G.n_v : G.n_u;
    const i64 n = wing ? G.m : a.nx;  // entities
    if (n == 0) return;
    i32 *eid_u = nullptr;
    if (wing) {
        // edge ids of the U-side entries are their slots
        eid_u = c.alloc<i32>(G.m);
        iota_i32(c, eid_u, G.m);
        a.xeid = eid_u;
        a.yeid = G.veid;
    }
    const int grid = (int)std::max<i64>(1, std::min<i64>(a.nx, 64));
    a.cnt = c.alloc<u32>((i64)grid * std::max<i64>(a.nx, 1));
    a.touch = c.alloc<i32>((i64)grid * std::max<i64>(a.nx, 1));
    a.e0 = wing ? c.alloc<i32>((i64)grid * std::max<i64>(a.nx, 1)) : nullptr;
    a.next = c.alloc<u32>(1);
    a.p = c.alloc<i32>(n);
    PBNG_HIP(hipMemsetAsync(a.cnt, 0, sizeof(u32) * grid * std::max<i64>(a.nx, 1), s));
    PBNG_HIP(hipMemsetAsync(a.next, 0, sizeof(u32), s));
    hipLaunchKernelGGL(h_init, dim3(grid_1d(n)), dim3(256), 0, s, a.p, n);
    if (a.nx > 0) hipLaunchKernelGGL(h_pairs, dim3(grid), dim3(HB), 0, s, a);
    hipLaunchKernelGGL(h_label, dim3(grid_1d(n)), dim3(256), 0, s, a.p, theta, k, n, comp);
    PBNG_LAUNCH_CHECK();
}

}  // namespace pbng
