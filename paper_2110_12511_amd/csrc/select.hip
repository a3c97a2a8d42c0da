// Range determination of the coarse-grained phase (Algorithm 4, find_range;
// Section 3.1.3).  Given the alive entities' supports (u64 keys) and work
// estimates, find the smallest support value s whose cumulative work
// sum{w_l : alive l, key_l <= s} reaches the target; when the alive work
// total is below the target, s is the largest alive support.  An optional
// count target also stops the range once the number of alive entities with
// key <= s reaches it (s is then the smaller of the two crossings), which
// bounds partitions made of many entities with little work each.
//
// Supports reach ~1e12 for tip decomposition, so bins per support value are
// not possible; the selection descends the key's bits 8 at a time (an
// MSB-first radix select with work-weighted 256-bin histograms).
#include "pbng_internal.h"

namespace pbng {

struct SelState {
    u64 total;     // alive work
    u64 maxkey;    // largest alive key
    u64 prefix;    // bits decided so far
    u64 rem;       // target still to cover inside the current prefix bucket
    u64 target;
    u64 result;    // s
    u64 work;      // cumulative work at s
    u64 done;      // 1 when the totals were below both targets (result = maxkey)
    u64 count;     // alive entities
    u64 rem_c;     // count target still to cover inside the bucket (~0: none)
};

// Per-block sum and maximum, then one pair of device atomics per block (a
// per-wave pair would queue thousands of same-address atomics).
__device__ __forceinline__ void block_sum_max(u64 t, u64 mx, u64 *sum_out, u64 *max_out) {
    __shared__ u64 s_t[256 / WAVE], s_m[256 / WAVE];
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        t += __shfl_down(t, d, WAVE);
        const u64 o = __shfl_down(mx, d, WAVE);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s_t[threadIdx.x / WAVE] = t;
        s_m[threadIdx.x / WAVE] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; ++i) {
            t += s_t[i];
            mx = s_m[i] > mx ? s_m[i] : mx;
        }
        if (t) atomicAdd((unsigned long long *)sum_out, (unsigned long long)t);
        if (max_out && mx) atomicMax((unsigned long long *)max_out, (unsigned long long)mx);
    }
}

__global__ __launch_bounds__(256) void k_sel_total(const u64 *key, const u64 *w, const unsigned char *state,
                                                  unsigned char alive, i64 n, SelState *st) {
    u64 t = 0, mx = 0, nc = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        if (state[i] != alive) continue;
        t += w[i];
        ++nc;
        u64 k = key[i];
        mx = k > mx ? k : mx;
    }
    block_sum_max(t, mx, &st->total, &st->maxkey);
    __syncthreads();
    block_sum_max(nc, 0, &st->count, nullptr);
}

// Target of the plain rule (Section 3.1.3): the alive work spread over the
// partitions still to create, times the scaling factor of the previous
// partition (ratio of its initial to its final work estimate).
__global__ void k_sel_init(SelState *st, const u64 *target, const double *scale, int parts_left, u64 count_target) {
    u64 tg;
    if (scale) {
        double t = (double)st->total / (double)(parts_left > 0 ? parts_left : 1) * scale[0];
        tg = t >= 1.8e19 ? ~0ull : (u64)t;
    } else {
        tg = *target;
    }
    if (tg == 0) tg = 1;
    st->target = tg;
    st->prefix = 0;
    st->rem = tg;
    st->rem_c = count_target ? count_target : ~0ull;
    if (st->total < tg && st->count < st->rem_c) {
        st->done = 1;
        st->result = st->maxkey;
        st->work = st->total;
    } else {
        st->done = 0;
    }
}

// work histogram in hist[0..255], count histogram in hist[256..511]
__global__ __launch_bounds__(256) void k_sel_hist(const u64 *key, const u64 *w, const unsigned char *state,
                                                 unsigned char alive, i64 n, int shift, const SelState *st, u64 *hist) {
    __shared__ u64 h[256];
    __shared__ u32 hc[256];
    h[threadIdx.x] = 0;
    hc[threadIdx.x] = 0;
    __syncthreads();
    // a level above the largest key's top bit has digit 0 for every key:
    // nothing to count (the pick keeps digit 0)
    if (!st->done && (st->maxkey >> shift) != 0) {
        const u64 pre = st->prefix;
        const int hs = shift + 8;
        for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
            if (state[i] != alive) continue;
            u64 k = key[i];
            if (hs < 64 && (k >> hs) != (pre >> hs)) continue;
            atomicAdd((unsigned long long *)&h[(k >> shift) & 255], (unsigned long long)w[i]);
            atomicAdd(&hc[(k >> shift) & 255], 1u);
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd((unsigned long long *)&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
    if (hc[threadIdx.x]) atomicAdd((unsigned long long *)&hist[256 + threadIdx.x], (unsigned long long)hc[threadIdx.x]);
}

// The smallest digit whose cumulative work covers the remaining target, or
// whose cumulative count covers the remaining count target, whichever comes
// first (256 threads, one digit each: inclusive prefixes in LDS, then the
// number of digits still below a target is its crossing); clears the
// histograms for the next level.
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, int shift, u64 *hist) {
    __shared__ u64 sh[256], sc[256];
    const int d = threadIdx.x;
    const u64 h = hist[d], hcnt = hist[256 + d];
    hist[d] = 0;
    hist[256 + d] = 0;
    if (st->done || (st->maxkey >> shift) == 0) return;  // block-uniform
    sh[d] = h;
    sc[d] = hcnt;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const u64 v = d >= off ? sh[d - off] : 0, vc = d >= off ? sc[d - off] : 0;
        __syncthreads();
        sh[d] += v;
        sc[d] += vc;
        __syncthreads();
    }
    const u64 rem = st->rem, rem_c = st->rem_c;
    const int below_w = __syncthreads_count(sh[d] < rem ? 1 : 0);
    const int below_c = __syncthreads_count(sc[d] < rem_c ? 1 : 0);
    if (d == 0) {
        const int pick = below_w < below_c ? below_w : below_c;
        if (pick < 256) {
            st->rem = rem - (pick ? sh[pick - 1] : 0);
            if (rem_c != ~0ull) st->rem_c = rem_c - (pick ? sc[pick - 1] : 0);
        }
        st->prefix |= (u64)(pick < 256 ? pick : 255) << shift;
    }
}

__global__ __launch_bounds__(256) void k_sel_work(const u64 *key, const u64 *w, const unsigned char *state,
                                                 unsigned char alive, i64 n, SelState *st) {
    if (st->done) return;
    const u64 s = st->prefix;
    u64 t = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        if (state[i] == alive && key[i] <= s) t += w[i];
    block_sum_max(t, 0, &st->work, nullptr);
}

__global__ void k_sel_finish(SelState *st, u64 *s_out, u64 *work_out) {
    if (!st->done) st->result = st->prefix;
    *s_out = st->result;
    if (work_out) *work_out = st->work;
}

static int grid_sel(i64 n) {
    i64 g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 512 ? 512 : g));
}

// All launches are asynchronous on the context stream; results stay on the
// device.  The number of 8-bit levels is fixed at 8 (full u64 keys) unless
// `key_bits` narrows it.
void weighted_select(Ctx &c, const u64 *key, const u64 *w, const unsigned char *state, unsigned char alive, i64 n,
                     const u64 *target_dev, const double *scale_dev, int parts_left, u64 *s_out,
                     u64 *work_at_s_out, u64 count_target) {
    if (!c.sel_scratch) PBNG_HIP(hipMalloc(&c.sel_scratch, sizeof(SelState) + 512 * sizeof(u64)));
    SelState *st = static_cast<SelState *>(c.sel_scratch);
    u64 *hist = reinterpret_cast<u64 *>(st + 1);
    PBNG_HIP(hipMemsetAsync(st, 0, sizeof(SelState), c.stream));
    PBNG_HIP(hipMemsetAsync(hist, 0, 512 * sizeof(u64), c.stream));
    hipLaunchKernelGGL(k_sel_total, dim3(grid_sel(n)), dim3(256), 0, c.stream, key, w, state, alive, n, st);
    PBNG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, c.stream, st, target_dev, scale_dev, parts_left, count_target);
    PBNG_LAUNCH_CHECK();
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(grid_sel(n)), dim3(256), 0, c.stream, key, w, state, alive, n, shift,
                           (const SelState *)st, hist);
        PBNG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, c.stream, st, shift, hist);
        PBNG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_sel_work, dim3(grid_sel(n)), dim3(256), 0, c.stream, key, w, state, alive, n, st);
    PBNG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_finish, dim3(1), dim3(1), 0, c.stream, st, s_out, work_at_s_out);
    PBNG_LAUNCH_CHECK();
}

}  // namespace pbng
