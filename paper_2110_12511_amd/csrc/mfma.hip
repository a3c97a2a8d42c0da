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

// Gram tiles.  The Gram matrix is symmetric, so only tiles (bi, bj) with
// bi <= bj of the 128 x 128 tiling are computed, and each count c(x, x')
// credits C(c, 2) to both hubs (on a diagonal tile, only entries above the
// diagonal).  A 256-lane workgroup owns one tile: per step it stages 128
// rows x 128 bytes of each operand in LDS (rows padded by 16 bytes against
// bank conflicts), loading the next step into registers while the matrix
// cores work on the current one, and wave w computes the 64 x 64 quarter
// (w / 2, w % 2) as 4 x 4 v_mfma_i32_16x16x64_i8 tiles.  v_mfma 16x16x64 i8:
// lane l feeds row (l % 16) with bytes 16 (l / 16) .. +15 of the 64-byte k
// chunk of A, and the same bytes of column (l % 16) of B; accumulator entry
// e of lane l is row 4 (l / 16) + e, column l % 16.  B = A_H^T, so both
// operands are hub rows.
constexpr int GT = 128;        // output tile
constexpr int GK = 128;        // k bytes per step (two 64-byte MFMA chunks)
constexpr int GROW = GK + 16;  // padded LDS row

__device__ __forceinline__ void gram_tile_of(u32 t, u32 nt, u32 &bi, u32 &bj) {
    // t-th pair (bi, bj), bi <= bj, in row-major order of the upper triangle
    u32 r = 0, rem = t;
    while (rem >= nt - r) {
        rem -= nt - r;
        ++r;
    }
    bi = r;
    bj = r + rem;
}

__global__ __launch_bounds__(256) void m_gram(const signed char *D, i64 kp, u32 h, const i32 *hubs, u64 *out,
                                             KCounters *kc) {
    __shared__ __attribute__((aligned(16))) signed char sA[GT * GROW];
    __shared__ __attribute__((aligned(16))) signed char sB[GT * GROW];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const u32 nt = (h + GT - 1) / GT;
    u32 bi, bj;
    gram_tile_of(blockIdx.x, nt, bi, bj);
    const i64 ra0 = (i64)bi * GT, rb0 = (i64)bj * GT;
    // staging: thread t loads 16-byte pieces (row t / 8 + 32 q, bytes 16 (t % 8))
    const int lr = threadIdx.x >> 3, lc = (threadIdx.x & 7) * 16;
    const v4i zero = {0, 0, 0, 0};
    v4i pa[4], pb[4];
    auto load = [&](i64 k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const i64 ra = ra0 + lr + 32 * q, rb = rb0 + lr + 32 * q;
            pa[q] = ra < h ? *reinterpret_cast<const v4i *>(D + ra * kp + k0 + lc) : zero;
            pb[q] = rb < h ? *reinterpret_cast<const v4i *>(D + rb * kp + k0 + lc) : zero;
        }
    };
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = zero;
    load(0);
    for (i64 k0 = 0; k0 < kp; k0 += GK) {
        __syncthreads();  // the previous step's reads of the LDS tiles are done
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<v4i *>(sA + (lr + 32 * q) * GROW + lc) = pa[q];
            *reinterpret_cast<v4i *>(sB + (lr + 32 * q) * GROW + lc) = pb[q];
        }
        __syncthreads();
        if (k0 + GK < kp) load(k0 + GK);
#pragma unroll
        for (int kc = 0; kc < GK; kc += 64) {
            v4i a[4], b[4];
            const int off = kc + 16 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = *reinterpret_cast<const v4i *>(sA + (wr + 16 * i + (lane & 15)) * GROW + off);
                b[i] = *reinterpret_cast<const v4i *>(sB + (wc + 16 * i + (lane & 15)) * GROW + off);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // C(c, 2) of every counted pair to both hubs: row sums over the lanes of
    // a row group, column sums over the lanes of a column
    u64 rs[4][4], cs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) cs[j] = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int e = 0; e < 4; ++e) rs[i][e] = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const i64 gc = rb0 + wc + 16 * j + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const i64 gr = ra0 + wr + 16 * i + 4 * (lane >> 4) + e;
                if (gr < h && gc < h && (bi < bj || gr < gc)) {
                    const u64 cc = (u64)(u32)acc[i][j][e];
                    const u64 v = cc * (cc - 1) / 2;
                    rs[i][e] += v;
                    cs[j] += v;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            u64 v = rs[i][e];
            for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d, WAVE);
            const i64 gr = ra0 + wr + 16 * i + 4 * (lane >> 4) + e;
            if ((lane & 15) == 0 && gr < h && v) atomicAdd((unsigned long long *)&out[hubs[gr]], (unsigned long long)v);
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        u64 v = cs[j];
        v += __shfl_xor(v, 16, WAVE);
        v += __shfl_xor(v, 32, WAVE);
        const i64 gc = rb0 + wc + 16 * j + (lane & 15);
        if (lane < 16 && gc < h && v) atomicAdd((unsigned long long *)&out[hubs[gc]], (unsigned long long)v);
    }
    // multiply-adds issued (2 ops each) and the operand bytes read
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&kc->wedges, (unsigned long long)(2ull * GT * GT * (u64)kp));
        atomicAdd((unsigned long long *)&kc->items, (unsigned long long)(2ull * GT * (u64)kp));
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
        const i64 kp = (ny + GK - 1) / GK * GK;
        signed char *D = c.alloc<signed char>((i64)h * kp);
        PBNG_HIP(hipMemsetAsync(D, 0, (size_t)h * kp, s));
        hipLaunchKernelGGL(m_densify, dim3(grid_1d((i64)h * WAVE)), dim3(256), 0, s, (const i32 *)hubs, (const u32 *)nh, xrow,
                           xadj, kp, D);
        PBNG_LAUNCH_CHECK();
        const u32 nt = (h + GT - 1) / GT;
        const u32 tiles = nt * (nt + 1) / 2;  // upper triangle
        c.kbegin(PBNG_K_DENSE);
        hipLaunchKernelGGL(m_gram, dim3(tiles), dim3(256), 0, s, (const signed char *)D, kp, h, (const i32 *)hubs, out,
                           c.kctr + PBNG_K_DENSE);
        c.kend(PBNG_K_DENSE);
        PBNG_LAUNCH_CHECK();
        c.stats.dense_pairs += (u64)h * (u64)(h - 1) / 2;
    }
    return w;
}

}  // namespace pbng
