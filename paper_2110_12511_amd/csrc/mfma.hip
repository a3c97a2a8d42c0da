// Hub blocks on matrix cores.
//
// For the hub set H of one side X (vertices of degree above a cut-over), the
// common-neighbour counts c(x, x') = |N_x ∩ N_x'| of all hub pairs are the
// Gram matrix A_H A_H^T of the 0/1 adjacency rows of the hubs, an exact
// int8 x int8 -> int32 contraction (every count is below 2^31).  Each hub
// then owns sum over other hubs x' of C(c(x, x'), 2): its butterflies whose
// other X vertex is a hub.  The traversal counts everything else
// (process_start_xside); the two parts add up to the per-vertex counts of
// Section 2.1.  The paper notes that wedges concentrate on a few high-degree
// vertices; this moves the hub-hub share of them onto MFMA tiles.
#include <algorithm>

#include "dev_common.h"
#include "pbng_internal.h"

namespace pbng {

typedef int v4i __attribute__((ext_vector_type(4)));

enum : unsigned char { MC_Y = 0, MC_X = 1, MC_XHUB = 2 };

// vertex classes by label and the list of hubs (X ids)
__global__ void m_classes(const i32 *gid, i64 n, i64 xoff, i64 nx, const i64 *xrow, i32 cut, unsigned char *lclass,
                          i32 *hubs, u32 *nh) {
    const i64 stride = (i64)gridDim.x * blockDim.x;
    const i64 nn = (n + WAVE - 1) / WAVE * WAVE;
    for (i64 l = blockIdx.x * (i64)blockDim.x + threadIdx.x; l < nn; l += stride) {
        bool hub = false;
        i64 x = -1;
        if (l < n) {
            x = (i64)gid[l] - xoff;
            unsigned char cl = MC_Y;
            if (x >= 0 && x < nx) {
                hub = (xrow[x + 1] - xrow[x]) > cut;
                cl = hub ? MC_XHUB : MC_X;
            }
            lclass[l] = cl;
        }
        const u32 p = wave_append(nh, hub);
        if (hub) hubs[p] = (i32)x;
    }
}

// dense 0/1 int8 rows of the hubs over all Y columns (row stride kp); one
// wave per hub
__global__ void m_densify(const i32 *hubs, const u32 *nh, const i64 *xrow, const i32 *xadj, i64 kp, signed char *D) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    const u32 h = *nh;
    for (i64 r = wave; r < h; r += nwaves) {
        const i32 x = hubs[r];
        signed char *row = D + r * kp;
        for (i64 j = xrow[x] + lane; j < xrow[x + 1]; j += WAVE) row[xadj[j]] = 1;
    }
}

// Gram tiles: a 256-lane workgroup owns a 64 x 64 output tile; wave w owns
// rows 16w..16w+15 of it as four 16 x 16 accumulators.  v_mfma 16x16x64 i8:
// lane l feeds row (l % 16) with bytes k0 + 16 (l / 16) .. +15 of A, and the
// same bytes of column (l % 16) of B; accumulator entry i of lane l is row
// 4 (l / 16) + i, column l % 16.  B = A_H^T, so both operands are hub rows.
// Each output row sums C(c, 2) over the other hubs and adds it to its hub.
__global__ __launch_bounds__(256) void m_gram(const signed char *D, i64 kp, u32 h, const i32 *hubs, u64 *out,
                                             KCounters *kc) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const i64 r0 = (i64)blockIdx.y * 64 + 16 * w;
    const i64 c0 = (i64)blockIdx.x * 64;
    const i64 arow = r0 + (lane & 15);
    const int kq = (lane >> 4) * 16;
    v4i acc[4];
    for (int b = 0; b < 4; ++b) acc[b] = (v4i){0, 0, 0, 0};
    const v4i zero = {0, 0, 0, 0};
    for (i64 k0 = 0; k0 < kp; k0 += 64) {
        const v4i a = arow < h ? *reinterpret_cast<const v4i *>(D + arow * kp + k0 + kq) : zero;
        for (int b = 0; b < 4; ++b) {
            const i64 bcol = c0 + 16 * b + (lane & 15);
            const v4i bv = bcol < h ? *reinterpret_cast<const v4i *>(D + bcol * kp + k0 + kq) : zero;
            acc[b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bv, acc[b], 0, 0, 0);
        }
    }
    u64 rs[4] = {0, 0, 0, 0};
    for (int b = 0; b < 4; ++b) {
        const i64 col = c0 + 16 * b + (lane & 15);
        for (int i = 0; i < 4; ++i) {
            const i64 row = r0 + 4 * (lane >> 4) + i;
            if (row < h && col < h && row != col) {
                const u64 cc = (u64)(u32)acc[b][i];
                rs[i] += cc * (cc - 1) / 2;
            }
        }
    }
    // rows are shared by the 16 lanes with the same lane / 16
    for (int i = 0; i < 4; ++i) {
        u64 v = rs[i];
        for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d, WAVE);
        const i64 row = r0 + 4 * (lane >> 4) + i;
        if ((lane & 15) == 0 && row < h && v) atomicAdd((unsigned long long *)&out[hubs[row]], (unsigned long long)v);
    }
    // multiply-adds issued (2 ops each) and the tile bytes read
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&kc->wedges, (unsigned long long)(2ull * 64 * 64 * (u64)kp));
        atomicAdd((unsigned long long *)&kc->items, (unsigned long long)(2ull * 64 * (u64)kp));
    }
}

u64 count_side(Ctx &c, const DevGraph &G, int side, const pbng_opts &o, u64 *out) {
    hipStream_t s = c.stream;
    const i64 nx = side == 0 ? G.n_u : G.n_v;
    const i64 ny = side == 0 ? G.n_v : G.n_u;
    const i64 xoff = side == 0 ? 0 : G.n_u;
    const i64 *xrow = side == 0 ? G.urow : G.vrow;
    const i32 *xadj = side == 0 ? G.ucol : G.vadj;
    const int cut = o.dense_cut == 0 ? 1024 : o.dense_cut;
    // the packed traversal counters need every count below 2^16
    const bool dense = !(o.flags & PBNG_F_NO_DENSE_TILE) && o.dense_cut >= 0 && G.maxdeg < 65536 && nx > 0;
    u64 *sl = c.alloc<u64>(G.n);
    if (!dense) {
        const u64 w = count_pass(c, G, sl, nullptr, nullptr);
        gather_side(c, G, sl, side, out);
        return w;
    }
    unsigned char *lclass = c.alloc<unsigned char>(G.n);
    i32 *hubs = c.alloc<i32>(nx);
    u32 *nh = c.alloc<u32>(1);
    PBNG_HIP(hipMemsetAsync(nh, 0, sizeof(u32), s));
    hipLaunchKernelGGL(m_classes, dim3(grid_1d(G.n)), dim3(256), 0, s, (const i32 *)G.gid, G.n, xoff, nx, xrow, cut, lclass,
                       hubs, nh);
    PBNG_LAUNCH_CHECK();
    const u32 h = read_scalar<u32>(c, nh);
    const u64 w = count_pass_xside(c, G, sl, lclass);
    gather_side(c, G, sl, side, out);
    if (h >= 2) {
        const i64 kp = (ny + 63) / 64 * 64;
        signed char *D = c.alloc<signed char>((i64)h * kp);
        PBNG_HIP(hipMemsetAsync(D, 0, (size_t)h * kp, s));
        hipLaunchKernelGGL(m_densify, dim3(grid_1d((i64)h * WAVE)), dim3(256), 0, s, (const i32 *)hubs, (const u32 *)nh, xrow,
                           xadj, kp, D);
        PBNG_LAUNCH_CHECK();
        const u32 tiles = (h + 63) / 64;
        c.kbegin(PBNG_K_DENSE);
        hipLaunchKernelGGL(m_gram, dim3(tiles, tiles), dim3(256), 0, s, (const signed char *)D, kp, h, (const i32 *)hubs, out,
                           c.kctr + PBNG_K_DENSE);
        c.kend(PBNG_K_DENSE);
        PBNG_LAUNCH_CHECK();
        c.stats.dense_pairs += (u64)h * (u64)(h - 1) / 2;
    }
    return w;
}

}  // namespace pbng
