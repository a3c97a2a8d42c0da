// Device primitives: exclusive scan, stable LSD radix sort (wave64 ballot
// ranking), fills and small reductions.  Plain building blocks for the
// preprocessing, binning and partitioning steps.
#include "pbng_internal.h"

namespace pbng {

// ------------------------------------------------------------------ arena

void *Arena::take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (fixed_base) {
        if (bytes > fixed_cap - fixed_used)
            throw Error(PBNG_E_NOMEM, "the no-allocation scratch of " + std::to_string(fixed_cap >> 20) +
                                          " MiB is too small for this graph (" + std::to_string(fixed_used + bytes) +
                                          " bytes needed so far)");
        void *p = fixed_base + fixed_used;
        fixed_used += bytes;
        return p;
    }
    auto it = free_blocks.lower_bound(bytes);
    if (it != free_blocks.end() && it->first <= 2 * bytes + (64u << 20)) {
        void *p = it->second;
        size_t sz = it->first;
        free_blocks.erase(it);
        in_use.push_back({p, sz});
        return p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        // drop cached blocks and retry once
        for (auto &kv : free_blocks) (void)hipFree(kv.second);
        bytes_held = 0;
        for (auto &b : in_use) bytes_held += b.second;
        free_blocks.clear();
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(PBNG_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
    bytes_held += bytes;
    in_use.push_back({p, bytes});
    return p;
}

void Arena::release_all() {
    fixed_used = 0;
    for (auto &b : in_use) free_blocks.insert({b.second, b.first});
    in_use.clear();
}

void Arena::release_to(size_t mark) {
    if (fixed_base) {
        if (mark < fixed_used) fixed_used = mark;
        return;
    }
    while (in_use.size() > mark) {
        free_blocks.insert({in_use.back().second, in_use.back().first});
        in_use.pop_back();
    }
}

void Arena::destroy() {
    release_all();
    for (auto &kv : free_blocks) (void)hipFree(kv.second);
    free_blocks.clear();
    bytes_held = 0;
}

// ------------------------------------------------------------------ kernel timing

hipEvent_t Ctx::event() {
    if (ev_next == ev_pool.size()) {
        hipEvent_t e;
        PBNG_HIP(hipEventCreate(&e));
        ev_pool.push_back(e);
    }
    return ev_pool[ev_next++];
}

// Histogram over small key ranges: every block accumulates in LDS and adds
// its bins to the output once, instead of one device-scope atomic per element
// on a handful of contended counters.
constexpr int HIST_LDS = 4096;

template <class T>
__global__ __launch_bounds__(256) void k_hist_add(const i32 *key, const T *val, i64 n, i32 nb, T *out) {
    __shared__ T h[HIST_LDS];
    if (nb <= HIST_LDS) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0;
        __syncthreads();
        for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
            atomicAdd(&h[key[i]], val ? val[i] : T(1));
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            if (h[b]) atomicAdd(&out[b], h[b]);
    } else {
        for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
            atomicAdd(&out[key[i]], val ? val[i] : T(1));
    }
}

void hist_add_u32(Ctx &c, const i32 *key, i64 n, i32 nb, u32 *out) {
    if (n <= 0) return;
    const int g = (int)std::min<i64>((n + 255) / 256, (i64)c.num_cu * 4);
    hipLaunchKernelGGL(k_hist_add<u32>, dim3(g), dim3(256), 0, c.stream, key, (const u32 *)nullptr, n, nb, out);
    PBNG_LAUNCH_CHECK();
}

void hist_add_u64(Ctx &c, const i32 *key, const u64 *val, i64 n, i32 nb, u64 *out) {
    if (n <= 0) return;
    const int g = (int)std::min<i64>((n + 255) / 256, (i64)c.num_cu * 4);
    hipLaunchKernelGGL(k_hist_add<unsigned long long>, dim3(g), dim3(256), 0, c.stream, key,
                       reinterpret_cast<const unsigned long long *>(val), n, nb, reinterpret_cast<unsigned long long *>(out));
    PBNG_LAUNCH_CHECK();
}

hipStream_t Ctx::capture_stream() {
    // non-blocking, default priority
    if (!cap_stream) PBNG_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    return cap_stream;
}

hipStream_t Ctx::aux() {
    if (!aux_stream) PBNG_HIP(hipStreamCreateWithFlags(&aux_stream, hipStreamNonBlocking));
    return aux_stream;
}

void Ctx::kbegin(int cls, hipStream_t st) {
    if (!timing) return;
    hipEvent_t a = event(), b = event();
    PBNG_HIP(hipEventRecord(a, st ? st : stream));
    intervals[cls].push_back({a, b});
}

void Ctx::kend(int cls, hipStream_t st) {
    if (!timing) return;
    PBNG_HIP(hipEventRecord(intervals[cls].back().second, st ? st : stream));
}

void Ctx::timing_begin_call(bool on) {
    timing = on;
    ev_next = 0;
    for (auto &v : intervals) v.clear();
    if (!kctr) PBNG_HIP(hipMalloc(&kctr, sizeof(KCounters) * PBNG_K_NCLASS));
    PBNG_HIP(hipMemsetAsync(kctr, 0, sizeof(KCounters) * PBNG_K_NCLASS, stream));
}

// Algorithmic bytes per unit of work:
//   traversal kernels: 4 B per wedge (the id of its far end), 12 B per list
//   segment (the middle vertex's id and its offset pair), 16 B per 64-bit
//   atomic update (read-modify-write), 16 B per item (its offsets and
//   support);
//   wing batch updates: 8 B per link walked (bloom id and twin), 16 B per
//   atomic support update, 16 B per bloom touched (bloom number, count and
//   offsets).
void Ctx::timing_end_call() {
    PBNG_HIP(hipStreamSynchronize(stream));
    KCounters h[PBNG_K_NCLASS];
    PBNG_HIP(hipMemcpy(h, kctr, sizeof(h), hipMemcpyDeviceToHost));
    for (int k = 0; k < PBNG_K_NCLASS; ++k) {
        pbng_kernel_stat &s = stats.kstat[k];
        s.ms = 0;
        s.launches = intervals[k].size();
        for (auto &iv : intervals[k]) {
            float ms = 0;
            PBNG_HIP(hipEventElapsedTime(&ms, iv.first, iv.second));
            s.ms += ms;
        }
        s.wedges = h[k].wedges;
        if (k == PBNG_K_WING_CD)
            s.bytes = 8 * h[k].wedges + 16 * h[k].atomics + 16 * h[k].segments + 16 * h[k].items;
        else if (k == PBNG_K_DENSE)
            s.bytes = h[k].items;  // int8 tile bytes; wedges holds the int8 ops

        else
            s.bytes = 4 * h[k].wedges + 12 * h[k].segments + 16 * h[k].atomics + 16 * h[k].items;
    }
    timing = false;
}

// ------------------------------------------------------------------ small kernels

template <class T>
__global__ void k_fill(T *p, T v, i64 n) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_iota(i32 *p, i64 n) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = (i32)i;
}

// Radix-sort width: bits needed for maxval, rounded up to whole bytes.
int bits_for(u64 maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return (b + 7) / 8 * 8;
}

int grid_1d(i64 n, int block, int cap) {
    i64 g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

static int grid_for(i64 n, int block = 256, int cap = 8192) {
    i64 g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <class T>
void fill(Ctx &c, T *p, T v, i64 n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, c.stream, p, v, n);
    PBNG_LAUNCH_CHECK();
}
template void fill<u64>(Ctx &, u64 *, u64, i64);
template void fill<i64>(Ctx &, i64 *, i64, i64);
template void fill<i32>(Ctx &, i32 *, i32, i64);
template void fill<u32>(Ctx &, u32 *, u32, i64);
template void fill<unsigned char>(Ctx &, unsigned char *, unsigned char, i64);

void iota_i32(Ctx &c, i32 *p, i64 n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, c.stream, p, n);
    PBNG_LAUNCH_CHECK();
}

template <class T>
T read_scalar(Ctx &c, const T *dev) {
    T h;
    PBNG_HIP(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, c.stream));
    PBNG_HIP(hipStreamSynchronize(c.stream));
    return h;
}
template u64 read_scalar<u64>(Ctx &, const u64 *);
template i64 read_scalar<i64>(Ctx &, const i64 *);
template u32 read_scalar<u32>(Ctx &, const u32 *);
template i32 read_scalar<i32>(Ctx &, const i32 *);

// ------------------------------------------------------------------ scan
// Three phases: per-tile totals, scan of the totals (recursive), tile scans
// with the carried prefix.  Tile = 256 threads x 8 items.

constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

template <class T>
__device__ T block_exclusive_scan(T v, T *sh, T &total) {
    // sh: SCAN_T / WAVE entries
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    T x = v;
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    if (lane == WAVE - 1) sh[wid] = x;
    __syncthreads();
    T off = 0, tot = 0;
    for (int w = 0; w < SCAN_T / WAVE; ++w) {
        if (w < wid) off += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

template <class T>
__global__ __launch_bounds__(SCAN_T) void k_tile_sums(const T *in, i64 n, T *sums) {
    __shared__ T sh[SCAN_T / WAVE];
    i64 base = (i64)blockIdx.x * SCAN_TILE;
    T s = 0;
    for (int k = 0; k < SCAN_I; ++k) {
        i64 i = base + (i64)k * SCAN_T + threadIdx.x;
        if (i < n) s += in[i];
    }
    T tot;
    block_exclusive_scan<T>(s, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(SCAN_T) void k_tile_scan(const T *in, i64 n, const T *carry, T *out) {
    __shared__ T sh[SCAN_T / WAVE];
    i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_I;
    T v[SCAN_I];
    T s = 0;
    for (int k = 0; k < SCAN_I; ++k) {
        i64 i = base + k;
        v[k] = i < n ? in[i] : T(0);
        s += v[k];
    }
    T tot;
    T run = block_exclusive_scan<T>(s, sh, tot) + (carry ? carry[blockIdx.x] : T(0));
    for (int k = 0; k < SCAN_I; ++k) {
        i64 i = base + k;
        if (i <= n) out[i] = run;  // out has n+1 entries
        run += v[k];
    }
}

template <class T>
void exclusive_scan(Ctx &c, const T *in, T *out, i64 n) {
    // out[i] = sum in[0..i), for i in [0, n]; out must hold n+1 entries.
    i64 ntiles = (n + 1 + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles <= 1) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(SCAN_T), 0, c.stream, in, n, (const T *)nullptr, out);
        PBNG_LAUNCH_CHECK();
        return;
    }
    T *sums = c.alloc<T>(ntiles);
    T *carry = c.alloc<T>(ntiles + 1);
    hipLaunchKernelGGL(k_tile_sums<T>, dim3(ntiles), dim3(SCAN_T), 0, c.stream, in, n, sums);
    PBNG_LAUNCH_CHECK();
    exclusive_scan<T>(c, sums, carry, ntiles);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(ntiles), dim3(SCAN_T), 0, c.stream, in, n, (const T *)carry, out);
    PBNG_LAUNCH_CHECK();
}
template void exclusive_scan<i64>(Ctx &, const i64 *, i64 *, i64);
template void exclusive_scan<u64>(Ctx &, const u64 *, u64 *, i64);
template void exclusive_scan<u32>(Ctx &, const u32 *, u32 *, i64);

// ------------------------------------------------------------------ reduce

__global__ __launch_bounds__(256) void k_sum_u64(const u64 *p, i64 n, u64 *out) {
    __shared__ u64 sh[4];
    u64 s = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) s += p[i];
    for (int d = WAVE / 2; d > 0; d >>= 1) s += __shfl_down(s, d, WAVE);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)out, (unsigned long long)(sh[0] + sh[1] + sh[2] + sh[3]));
}

u64 reduce_sum_u64(Ctx &c, const u64 *p, i64 n) {
    u64 *o = c.alloc<u64>(1);
    PBNG_HIP(hipMemsetAsync(o, 0, sizeof(u64), c.stream));
    if (n > 0) {
        hipLaunchKernelGGL(k_sum_u64, dim3(grid_for(n, 256, 1024)), dim3(256), 0, c.stream, p, n, o);
        PBNG_LAUNCH_CHECK();
    }
    return read_scalar<u64>(c, o);
}

// ------------------------------------------------------------------ radix sort
// Stable LSD sort of (u64 key, i32 value) pairs on the low `bits` bits, 8 bits
// per pass.  Each tile of RS_TILE items builds a digit histogram; a scan over
// the digit-major histogram matrix gives every (digit, tile) its output
// start; the scatter pass ranks items of equal digit inside a tile in input
// order, 256 at a time, using wave64 ballots to find equal-digit lanes.

constexpr int RS_T = 256, RS_R = 16, RS_TILE = RS_T * RS_R, RS_BINS = 256;

__global__ __launch_bounds__(RS_T) void k_rs_hist(const u64 *keys, i64 n, int shift, u32 *hist, i64 ntiles) {
    __shared__ u32 h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    i64 base = (i64)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_R; ++r) {
        i64 i = base + (i64)r * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(i64)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_T) void k_rs_scatter(const u64 *keys, const i32 *vals, i64 n, int shift,
                                                    const u32 *offs, i64 ntiles, u64 *okeys, i32 *ovals) {
    __shared__ u32 running[RS_BINS];
    __shared__ u32 wcnt[RS_T / WAVE][RS_BINS];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    running[tid] = offs[(i64)tid * ntiles + blockIdx.x];
    for (int w = 0; w < RS_T / WAVE; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const u64 lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    i64 base = (i64)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_R; ++r) {
        i64 i = base + (i64)r * RS_T + tid;
        bool valid = i < n;
        u64 k = valid ? keys[i] : 0;
        i32 v = (valid && vals) ? vals[i] : 0;
        u32 d = (u32)((k >> shift) & 0xFF);
        u64 peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            u64 bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        u32 rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            u32 before = 0;
            for (int w = 0; w < wid; ++w) before += wcnt[w][d];
            u32 pos = running[d] + before + rank;
            okeys[pos] = k;
            if (vals) ovals[pos] = v;
        }
        __syncthreads();
        u32 add = 0;
        for (int w = 0; w < RS_T / WAVE; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        running[tid] += add;
        __syncthreads();
    }
}

void radix_sort_u64(Ctx &c, u64 *keys, i32 *vals, i64 n, int bits, u64 **keys_out, i32 **vals_out) {
    *keys_out = keys;
    if (vals_out) *vals_out = vals;
    if (n <= 1 || bits <= 0) return;
    if (n >= (i64(1) << 32) - 1) throw Error(PBNG_E_OVERFLOW, "radix sort size beyond 2^32");
    i64 ntiles = (n + RS_TILE - 1) / RS_TILE;
    u32 *hist = c.alloc<u32>(ntiles * RS_BINS);
    u32 *offs = c.alloc<u32>(ntiles * RS_BINS + 1);
    u64 *k2 = c.alloc<u64>(n);
    i32 *v2 = vals ? c.alloc<i32>(n) : nullptr;
    u64 *ka = keys, *kb = k2;
    i32 *va = vals, *vb = v2;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(RS_T), 0, c.stream, (const u64 *)ka, n, shift, hist, ntiles);
        PBNG_LAUNCH_CHECK();
        exclusive_scan<u32>(c, hist, offs, ntiles * RS_BINS);
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(RS_T), 0, c.stream, (const u64 *)ka, (const i32 *)va, n,
                           shift, (const u32 *)offs, ntiles, kb, vb);
        PBNG_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *keys_out = ka;
    if (vals_out) *vals_out = va;
}

}  // namespace pbng
