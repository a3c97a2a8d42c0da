// Graph preprocessing (Algorithm 1, priority assignment and sorted lists).
//
// Vertices of W = U u V get labels in decreasing order of degree (ties by
// increasing global id, U ids before V ids), every adjacency list is sorted by
// increasing label, and for every directed entry (start -> mid) the number of
// wedge ends `last` in N_mid with label below both start and mid is stored:
// the wedges start -> mid -> last that the counting loop of Algorithm 1 walks
// form exactly that prefix of the sorted N_mid.
#include "pbng_internal.h"

namespace pbng {

// Row of CSR slot e: the last u with row[u] <= e (rows may be empty).
__device__ inline i64 row_of(const i64 *row, i64 n_u, i64 e) {
    i64 a = 0, b = n_u;  // answer in [0, n_u)
    while (a < b) {
        i64 c = (a + b + 1) >> 1;
        if (row[c] <= e) a = c; else b = c - 1;
    }
    return a;
}

__global__ void k_validate(i64 n_u, i64 n_v, i64 m, const i64 *row, const i32 *col, int *bad) {
    i64 stride = (i64)gridDim.x * blockDim.x;
    for (i64 u = blockIdx.x * (i64)blockDim.x + threadIdx.x; u < n_u; u += stride)
        if (row[u + 1] < row[u]) atomicOr(bad, 1);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (row[0] != 0 || row[n_u] != m)) atomicOr(bad, 1);
}

// edges are checked only once the row pointers are known to be sound
__global__ void k_validate_edges(i64 n_u, i64 n_v, i64 m, const i64 *row, const i32 *col, int *bad) {
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        i32 v = col[e];
        if (v < 0 || v >= n_v) { atomicOr(bad, 1); continue; }
        i64 u = row_of(row, n_u, e);
        if (e > row[u] && v <= col[e - 1]) atomicOr(bad, 1);
    }
}

__global__ void k_degrees(i64 n_u, i64 m, const i64 *row, const i32 *col, i32 *deg) {
    i64 stride = (i64)gridDim.x * blockDim.x;
    for (i64 u = blockIdx.x * (i64)blockDim.x + threadIdx.x; u < n_u; u += stride) deg[u] = (i32)(row[u + 1] - row[u]);
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += stride) atomicAdd(&deg[n_u + col[e]], 1);
}

__global__ void k_max_i32(const i32 *p, i64 n, i32 *out) {
    i32 mx = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) mx = max(mx, p[i]);
    for (int d = WAVE / 2; d > 0; d >>= 1) mx = max(mx, __shfl_down(mx, d, WAVE));
    if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

__global__ void k_vdeg64(i64 n_u, i64 n_v, const i32 *deg, i64 *vdeg) {
    for (i64 v = blockIdx.x * (i64)blockDim.x + threadIdx.x; v < n_v; v += (i64)gridDim.x * blockDim.x) vdeg[v] = deg[n_u + v];
}

__global__ void k_vkeys(i64 m, const i32 *col, u64 *keys, i32 *vals) {
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        keys[e] = (u64)col[e];
        vals[e] = (i32)e;
    }
}

__global__ void k_vscatter(i64 n_u, i64 m, const i64 *row, const i32 *veid, i32 *vadj) {
    for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < m; p += (i64)gridDim.x * blockDim.x)
        vadj[p] = (i32)row_of(row, n_u, veid[p]);
}

__global__ void k_deg_keys(const i32 *deg, i64 n, i32 maxdeg, u64 *keys) {
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < n; x += (i64)gridDim.x * blockDim.x)
        keys[x] = (u64)(maxdeg - deg[x]);
}

__global__ void k_labels(const i32 *gid, i64 n, const i32 *deg, i32 *label, i64 *degl) {
    for (i64 l = blockIdx.x * (i64)blockDim.x + threadIdx.x; l < n; l += (i64)gridDim.x * blockDim.x) {
        i32 x = gid[l];
        label[x] = (i32)l;
        degl[l] = deg[x];
    }
}

__global__ void k_pair_keys(i64 n_u, i64 n, i64 m, const i64 *row, const i32 *col, const i32 *label, u64 *keys, i32 *vals) {
    for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        i64 u = row_of(row, n_u, e);
        u64 lu = (u64)label[u];
        u64 lv = (u64)label[n_u + col[e]];
        keys[2 * e] = lu * (u64)n + lv;
        vals[2 * e] = (i32)e;
        keys[2 * e + 1] = lv * (u64)n + lu;
        vals[2 * e + 1] = (i32)e;
    }
}

__global__ void k_unpack_pairs(const u64 *keys, const i32 *vals, i64 cnt, i64 n, i32 *ladj, i32 *leid, i32 *lrow) {
    for (i64 j = blockIdx.x * (i64)blockDim.x + threadIdx.x; j < cnt; j += (i64)gridDim.x * blockDim.x) {
        u64 k = keys[j];
        ladj[j] = (i32)(k % (u64)n);
        lrow[j] = (i32)(k / (u64)n);
        leid[j] = vals[j];
    }
}

// lpl[j] for entry j = (start -> mid): |{last in N_mid : last < min(start, mid)}|,
// found by binary search in the sorted N_mid.
__global__ void k_prefix_len(const i32 *lrow, const i32 *ladj, const i64 *loff, i64 cnt, i32 *lpl, i64 *lpl64) {
    for (i64 j = blockIdx.x * (i64)blockDim.x + threadIdx.x; j < cnt; j += (i64)gridDim.x * blockDim.x) {
        i32 s = lrow[j], mid = ladj[j];
        i32 t = s < mid ? s : mid;
        i64 lo = loff[mid], hi = loff[mid + 1];
        i64 a = lo, b = hi;
        while (a < b) {
            i64 c = (a + b) >> 1;
            if (ladj[c] < t) a = c + 1; else b = c;
        }
        lpl[j] = (i32)(a - lo);
        lpl64[j] = a - lo;
    }
}

__global__ void k_row_sums(const i64 *pre, const i64 *loff, i64 n, i64 *wsum_rows) {
    for (i64 s = blockIdx.x * (i64)blockDim.x + threadIdx.x; s < n; s += (i64)gridDim.x * blockDim.x)
        wsum_rows[s] = pre[loff[s + 1]] - pre[loff[s]];
}

static int gridN(i64 n) {
    i64 g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}


void build_graph(Ctx &c, const pbng_csr &g, DevGraph &G) {
    G.n_u = g.n_u;
    G.n_v = g.n_v;
    G.n = g.n_u + g.n_v;
    G.m = g.m;
    G.urow = g.row_ptr;
    G.ucol = g.col_idx;
    const i64 n = G.n, m = G.m, n_u = G.n_u, n_v = G.n_v;
    hipStream_t s = c.stream;

    int *bad = c.alloc<int>(1);
    PBNG_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_validate, dim3(gridN(n_u > 0 ? n_u : 1)), dim3(256), 0, s, n_u, n_v, m, G.urow, G.ucol, bad);
    PBNG_LAUNCH_CHECK();
    if (read_scalar<i32>(c, bad)) throw Error(PBNG_E_GRAPH, "malformed CSR row pointers");
    if (m) {
        hipLaunchKernelGGL(k_validate_edges, dim3(gridN(m)), dim3(256), 0, s, n_u, n_v, m, G.urow, G.ucol, bad);
        PBNG_LAUNCH_CHECK();
        if (read_scalar<i32>(c, bad)) throw Error(PBNG_E_GRAPH, "malformed CSR (unsorted row, duplicate or out-of-range id)");
    }

    i32 *deg = c.alloc<i32>(n);
    PBNG_HIP(hipMemsetAsync(deg, 0, sizeof(i32) * (n ? n : 1), s));
    hipLaunchKernelGGL(k_degrees, dim3(gridN(m > n_u ? m : n_u)), dim3(256), 0, s, n_u, m, G.urow, G.ucol, deg);
    PBNG_LAUNCH_CHECK();

    // V-side CSR (U ids and edge ids)
    i64 *vdeg = c.alloc<i64>(n_v);
    G.vrow = c.alloc<i64>(n_v + 1);
    if (n_v) {
        hipLaunchKernelGGL(k_vdeg64, dim3(gridN(n_v)), dim3(256), 0, s, n_u, n_v, (const i32 *)deg, vdeg);
        PBNG_LAUNCH_CHECK();
    }
    exclusive_scan<i64>(c, vdeg, G.vrow, n_v);
    G.vadj = c.alloc<i32>(m);
    if (m) {
        // stable sort of edge ids by V id: every V list comes out in
        // increasing U id (the U-side CSR is u-major)
        u64 *vk = c.alloc<u64>(m);
        i32 *ve = c.alloc<i32>(m);
        hipLaunchKernelGGL(k_vkeys, dim3(gridN(m)), dim3(256), 0, s, m, G.ucol, vk, ve);
        PBNG_LAUNCH_CHECK();
        u64 *svk;
        radix_sort_u64(c, vk, ve, m, bits_for((u64)(n_v > 0 ? n_v - 1 : 0)), &svk, &G.veid);
        hipLaunchKernelGGL(k_vscatter, dim3(gridN(m)), dim3(256), 0, s, n_u, m, G.urow, (const i32 *)G.veid, G.vadj);
        PBNG_LAUNCH_CHECK();
    } else {
        G.veid = c.alloc<i32>(1);
    }

    // labels: stable sort of global ids by decreasing degree
    i32 *dmax = c.alloc<i32>(1);
    PBNG_HIP(hipMemsetAsync(dmax, 0, sizeof(i32), s));
    if (n) {
        hipLaunchKernelGGL(k_max_i32, dim3(gridN(n)), dim3(256), 0, s, (const i32 *)deg, n, dmax);
        PBNG_LAUNCH_CHECK();
    }
    i32 maxdeg = read_scalar<i32>(c, dmax);
    G.maxdeg = maxdeg;
    u64 *dkeys = c.alloc<u64>(n);
    i32 *ids = c.alloc<i32>(n);
    if (n) {
        hipLaunchKernelGGL(k_deg_keys, dim3(gridN(n)), dim3(256), 0, s, (const i32 *)deg, n, maxdeg, dkeys);
        PBNG_LAUNCH_CHECK();
    }
    iota_i32(c, ids, n);
    u64 *sk;
    i32 *sv;
    radix_sort_u64(c, dkeys, ids, n, bits_for((u64)maxdeg), &sk, &sv);
    G.gid = sv;
    G.label = c.alloc<i32>(n);
    i64 *degl = c.alloc<i64>(n);
    if (n) {
        hipLaunchKernelGGL(k_labels, dim3(gridN(n)), dim3(256), 0, s, (const i32 *)G.gid, n, (const i32 *)deg, G.label, degl);
        PBNG_LAUNCH_CHECK();
    }
    G.loff = c.alloc<i64>(n + 1);
    exclusive_scan<i64>(c, degl, G.loff, n);

    // sorted label adjacency of both sides
    const i64 cnt = 2 * m;
    u64 *pk = c.alloc<u64>(cnt);
    i32 *pv = c.alloc<i32>(cnt);
    if (m) {
        hipLaunchKernelGGL(k_pair_keys, dim3(gridN(m)), dim3(256), 0, s, n_u, n, m, G.urow, G.ucol, (const i32 *)G.label, pk, pv);
        PBNG_LAUNCH_CHECK();
    }
    u64 *spk;
    i32 *spv;
    radix_sort_u64(c, pk, pv, cnt, n > 1 ? bits_for((u64)n * (u64)n - 1) : 8, &spk, &spv);
    G.ladj = c.alloc<i32>(cnt);
    G.leid = c.alloc<i32>(cnt);
    i32 *lrow = c.alloc<i32>(cnt);
    G.lpl = c.alloc<i32>(cnt);
    i64 *lpl64 = c.alloc<i64>(cnt);
    if (cnt) {
        hipLaunchKernelGGL(k_unpack_pairs, dim3(gridN(cnt)), dim3(256), 0, s, (const u64 *)spk, (const i32 *)spv, cnt, n,
                           G.ladj, G.leid, lrow);
        PBNG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_prefix_len, dim3(gridN(cnt)), dim3(256), 0, s, (const i32 *)lrow, (const i32 *)G.ladj,
                           (const i64 *)G.loff, cnt, G.lpl, lpl64);
        PBNG_LAUNCH_CHECK();
    }
    i64 *pre = c.alloc<i64>(cnt + 1);
    exclusive_scan<i64>(c, lpl64, pre, cnt);
    G.wsum = c.alloc<i64>(n + 1);
    if (n) {
        hipLaunchKernelGGL(k_row_sums, dim3(gridN(n)), dim3(256), 0, s, (const i64 *)pre, (const i64 *)G.loff, n, G.wsum);
        PBNG_LAUNCH_CHECK();
    }
}

}  // namespace pbng
