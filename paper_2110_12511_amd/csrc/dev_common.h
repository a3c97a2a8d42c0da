// Device helpers shared by the traversal kernels: block scans and sums for
// wave64 workgroups, and the two wedge-count accumulators (an LDS hash and a
// dense HBM array with a touched list).
#pragma once

#include "pbng_internal.h"

namespace pbng {

__device__ __forceinline__ u64 ld_coherent(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ i64 ld_coherent(const i64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_coherent(const u32 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ i32 ld_coherent(const i32 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned char ld_coherent(const unsigned char *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_coherent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated append: one atomic per wave; returns this lane's slot
// (meaningful only where pred holds).  Call from every lane of the wave
// that reaches it.
__device__ __forceinline__ u32 wave_append(u32 *ctr, bool pred) {
    const u64 m = __ballot(pred);
    if (!m) return 0;
    const int lane = threadIdx.x & (WAVE - 1);
    const int leader = __ffsll((unsigned long long)m) - 1;
    u32 base = 0;
    if (lane == leader) base = atomicAdd(ctr, (u32)__popcll(m));
    base = __shfl(base, leader, WAVE);
    const u64 below = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    return base + (u32)__popcll(m & below);
}

// Per-thread tallies of algorithmic work, flushed once per workgroup.
struct Tally {
    u64 wedges = 0, segments = 0, atomics = 0, items = 0;
    __device__ void flush(KCounters *kc, u64 *wedges_out) {
        if (wedges) {
            if (wedges_out) atomicAdd((unsigned long long *)wedges_out, (unsigned long long)wedges);
            if (kc) atomicAdd((unsigned long long *)&kc->wedges, (unsigned long long)wedges);
        }
        if (kc && segments) atomicAdd((unsigned long long *)&kc->segments, (unsigned long long)segments);
        if (kc && atomics) atomicAdd((unsigned long long *)&kc->atomics, (unsigned long long)atomics);
        if (kc && items) atomicAdd((unsigned long long *)&kc->items, (unsigned long long)items);
    }
};

__device__ __forceinline__ u32 hash32(u32 x) { return x * 2654435761u; }

template <int BLOCK>
__device__ __forceinline__ i32 block_incl_scan_i32(i32 v, i32 *sh_wave, i32 &total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    i32 x = v;
    for (int d = 1; d < WAVE; d <<= 1) {
        i32 y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    if (BLOCK == WAVE) {
        total = __shfl(x, WAVE - 1, WAVE);
        return x;
    }
    if (lane == WAVE - 1) sh_wave[wid] = x;
    __syncthreads();
    i32 off = 0, tot = 0;
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        i32 t = sh_wave[w];
        if (w < wid) off += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return x + off;
}

template <int BLOCK>
__device__ __forceinline__ u64 block_min_u64(u64 v, u64 *sh) {
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        u64 o = __shfl_down(v, d, WAVE);
        v = o < v ? o : v;
    }
    if (BLOCK == WAVE) return __shfl(v, 0, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    u64 t = ~0ull;
    for (int w = 0; w < BLOCK / WAVE; ++w) t = sh[w] < t ? sh[w] : t;
    __syncthreads();
    return t;
}

template <int BLOCK>
__device__ __forceinline__ u64 block_sum_u64(u64 v, u64 *sh) {
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_down(v, d, WAVE);
    if (BLOCK == WAVE) return __shfl(v, 0, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    u64 t = 0;
    for (int w = 0; w < BLOCK / WAVE; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// ------------------------------------------------------------------ accumulators
// Both expose: add(key); entries(); entry(i, key, cnt) (key < 0: empty);
// handle(i) of entry i; find(key) -> handle; cnt(h); set_cnt(h, v);
// inc(h) (atomic, returns old); set_bid(h, b); bid(h); reset(tid).

// Open-addressing hash in LDS, linear probing, key -1 = empty.
struct LdsAcc {
    i32 *keys;
    u32 *vals;
    i32 *bids;
    u32 mask;
    int shift;
    __device__ void init(int logcap, int tid, int nthreads) {
        mask = (1u << logcap) - 1;
        shift = 32 - logcap;
        for (u32 i = tid; i <= mask; i += nthreads) {
            keys[i] = -1;
            vals[i] = 0;
        }
    }
    __device__ __forceinline__ void add(i32 key, u32 inc = 1u) {
        // each probe is one compare-and-swap: it claims an empty slot or
        // returns the slot's key (one LDS round trip per probe)
        u32 h = hash32((u32)key) >> shift;
        for (;;) {
            const i32 prev = atomicCAS(&keys[h], -1, key);
            if (prev == -1 || prev == key) break;
            h = (h + 1) & mask;
        }
        atomicAdd(&vals[h], inc);
    }
    __device__ __forceinline__ i64 entries() const { return (i64)mask + 1; }
    __device__ __forceinline__ void entry(i64 i, i32 &key, u32 &c) const {
        key = keys[i];
        c = vals[i];
    }
    __device__ __forceinline__ u32 handle(i64 i) const { return (u32)i; }
    __device__ __forceinline__ u32 find(i32 key) const {
        u32 h = hash32((u32)key) >> shift;
        while (keys[h] != key) h = (h + 1) & mask;
        return h;
    }
    __device__ __forceinline__ u32 cnt(u32 h) const { return vals[h]; }
    __device__ __forceinline__ void set_cnt(u32 h, u32 v) { vals[h] = v; }
    __device__ __forceinline__ u32 inc(u32 h) { return atomicAdd(&vals[h], 1u); }
    __device__ __forceinline__ void set_bid(u32 h, i32 b) { bids[h] = b; }
    __device__ __forceinline__ i32 bid(u32 h) const { return bids[h]; }
    __device__ void reset(int, int) {}
};

// Dense counters over all labels in HBM with a touched list.  All accesses
// are device-coherent (atomics or relaxed atomic loads/stores) so no stale
// line in the CU's vector cache is ever read.
struct DenseAcc {
    u32 *c;
    i32 *bids;
    i32 *touch;
    u32 *ntouch;
    __device__ __forceinline__ void add(i32 key, u32 inc = 1u) {
        u32 old = atomicAdd(&c[key], inc);
        if (old == 0) {
            u32 t = atomicAdd(ntouch, 1u);
            __hip_atomic_store(&touch[t], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __device__ __forceinline__ i64 entries() const {
        return (i64)__hip_atomic_load(ntouch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void entry(i64 i, i32 &key, u32 &cc) const {
        key = __hip_atomic_load(&touch[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cc = __hip_atomic_load(&c[key], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ u32 handle(i64 i) const {
        return (u32)__hip_atomic_load(&touch[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ u32 find(i32 key) const { return (u32)key; }
    __device__ __forceinline__ u32 cnt(u32 h) const {
        return __hip_atomic_load(&c[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void set_cnt(u32 h, u32 v) {
        __hip_atomic_store(&c[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ u32 inc(u32 h) { return atomicAdd(&c[h], 1u); }
    __device__ __forceinline__ void set_bid(u32 h, i32 b) {
        __hip_atomic_store(&bids[h], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ i32 bid(u32 h) const {
        return __hip_atomic_load(&bids[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void reset(int tid, int nthreads) {
        i64 nt = entries();
        for (i64 i = tid; i < nt; i += nthreads) set_cnt(handle(i), 0u);
        __syncthreads();
        if (tid == 0) __hip_atomic_store(ntouch, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
};

}  // namespace pbng
