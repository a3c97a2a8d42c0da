// Many graphs per launch.
//
// A butterfly lies inside one connected component, so the tip and wing
// numbers of a disjoint union of graphs are those of each graph.  A batch is
// therefore packed into one union graph (U ids, V ids and edge ids of graph g
// shifted by the totals of the graphs before it) and decomposed once: every
// counting pass, every coarse-grained round and the single persistent
// fine-grained launch serve all graphs of the batch together, and the
// fine-grained queue holds partitions of every graph.  Graphs are grouped into
// consecutive chunks of at most a given number of edges to bound the memory
// of one union.
#include <string>
#include <vector>

#include "pbng_internal.h"

namespace pbng {

namespace {

struct PackDesc {
    const i64 *rp;
    const i32 *ci;
    i64 n_u, n_v, m;
    i64 u_off, v_off, m_off;
};

// Every entry is checked against its own sizes before packing: a column id
// at or above the entry's n_v would otherwise land in the next graph's V
// range, and the union alone could not tell.  Row pointers first (one
// workgroup per graph; bad[0] = lowest failing entry)...
__global__ void k_check_rows(const PackDesc *d, int ng, int *bad) {
    for (int g = blockIdx.x; g < ng; g += gridDim.x) {
        const PackDesc x = d[g];
        bool ok = true;
        if (threadIdx.x == 0) ok = x.rp[0] == 0 && x.rp[x.n_u] == x.m;
        for (i64 i = threadIdx.x; ok && i < x.n_u; i += blockDim.x) ok = x.rp[i + 1] >= x.rp[i];
        if (!ok) atomicMin(bad, g);
    }
}

// ... then, with sound rows, every edge: id in [0, n_v) and strictly above
// its predecessor in the same row
__global__ void k_check_edges(const PackDesc *d, int ng, int *bad) {
    for (int g = blockIdx.x; g < ng; g += gridDim.x) {
        const PackDesc x = d[g];
        bool ok = true;
        for (i64 e = threadIdx.x; ok && e < x.m; e += blockDim.x) {
            const i32 v = x.ci[e];
            if (v < 0 || (i64)v >= x.n_v) {
                ok = false;
                break;
            }
            i64 a = 0, b = x.n_u;  // row of slot e: the last u with rp[u] <= e
            while (a < b) {
                const i64 c = (a + b + 1) >> 1;
                if (x.rp[c] <= e) a = c; else b = c - 1;
            }
            if (e > x.rp[a] && v <= x.ci[e - 1]) ok = false;
        }
        if (!ok) atomicMin(bad, g);
    }
}

// host entries: the same checks; returns the first failing entry or -1
int check_entries_host(const std::vector<PackDesc> &pd) {
    for (size_t g = 0; g < pd.size(); ++g) {
        const PackDesc &x = pd[g];
        if (x.rp[0] != 0 || x.rp[x.n_u] != x.m) return (int)g;
        for (i64 u = 0; u < x.n_u; ++u) {
            if (x.rp[u + 1] < x.rp[u]) return (int)g;
            for (i64 e = x.rp[u]; e < x.rp[u + 1]; ++e) {
                const i32 v = x.ci[e];
                if (v < 0 || (i64)v >= x.n_v || (e > x.rp[u] && v <= x.ci[e - 1])) return (int)g;
            }
        }
    }
    return -1;
}

// one workgroup per graph (grid-stride over graphs)
__global__ void k_pack(const PackDesc *d, int ng, i64 *prp, i32 *pci) {
    for (int g = blockIdx.x; g < ng; g += gridDim.x) {
        const PackDesc x = d[g];
        for (i64 i = threadIdx.x; i < x.n_u; i += blockDim.x) prp[x.u_off + i] = x.rp[i] + x.m_off;
        for (i64 j = threadIdx.x; j < x.m; j += blockDim.x) pci[x.m_off + j] = x.ci[j] + (i32)x.v_off;
    }
}

struct OutDesc {
    u64 *out;
    i64 off, n;
};

__global__ void k_unpack(const OutDesc *d, int ng, const u64 *src) {
    for (int g = blockIdx.x; g < ng; g += gridDim.x) {
        const OutDesc x = d[g];
        for (i64 i = threadIdx.x; i < x.n; i += blockDim.x) x.out[i] = src[x.off + i];
    }
}

}  // namespace

i64 batch_chunk_end(const pbng_csr *g, int ng, int first, i64 max_m) {
    // graphs [first, end) with at most max_m edges in total (at least one)
    i64 tot = 0;
    int e = first;
    while (e < ng) {
        if (e > first && tot + g[e].m > max_m) break;
        tot += g[e].m;
        ++e;
    }
    return e;
}

// Decomposes graphs [first, last) packed into one union.  kind 0: tip of
// `side`, kind 1: wing.
void batch_run(Ctx &c, const pbng_csr *g, int first, int last, int kind, int side, const pbng_opts &o,
               uint64_t *const *outs) {
    hipStream_t s = c.stream;
    const int ng = last - first;
    const bool on_dev = g[first].on_device != 0;
    i64 NU = 0, NV = 0, M = 0;
    std::vector<PackDesc> pd(ng);
    for (int k = 0; k < ng; ++k) {
        const pbng_csr &x = g[first + k];
        pd[k] = PackDesc{x.row_ptr, x.col_idx, x.n_u, x.n_v, x.m, NU, NV, M};
        NU += x.n_u;
        NV += x.n_v;
        M += x.m;
    }
    if (NU + NV >= (i64(1) << 31) - 1 || M >= (i64(1) << 30))
        throw Error(PBNG_E_OVERFLOW, "batch chunk exceeds the single-graph size limits");
    i64 *prp = c.alloc<i64>(NU + 1);
    i32 *pci = c.alloc<i32>(M);
    auto bad_entry = [&](int k) {
        return Error(PBNG_E_GRAPH, "batch entry " + std::to_string(first + k) +
                                       ": malformed CSR (row pointers, unsorted row, duplicate or out-of-range id)");
    };
    if (on_dev) {
        PackDesc *dd = c.alloc<PackDesc>(ng);
        PBNG_HIP(hipMemcpy(dd, pd.data(), sizeof(PackDesc) * ng, hipMemcpyHostToDevice));
        int *bad = c.alloc<int>(1);
        const int none = 0x7FFFFFFF;
        PBNG_HIP(hipMemcpyAsync(bad, &none, sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_check_rows, dim3(std::min(ng, 4096)), dim3(256), 0, s, (const PackDesc *)dd, ng, bad);
        PBNG_LAUNCH_CHECK();
        int b = read_scalar<int>(c, bad);
        if (b != none) throw bad_entry(b);
        hipLaunchKernelGGL(k_check_edges, dim3(std::min(ng, 4096)), dim3(256), 0, s, (const PackDesc *)dd, ng, bad);
        PBNG_LAUNCH_CHECK();
        b = read_scalar<int>(c, bad);
        if (b != none) throw bad_entry(b);
        hipLaunchKernelGGL(k_pack, dim3(std::min(ng, 4096)), dim3(256), 0, s, (const PackDesc *)dd, ng, prp, pci);
        PBNG_LAUNCH_CHECK();
        PBNG_HIP(hipMemcpyAsync(prp + NU, &M, sizeof(i64), hipMemcpyHostToDevice, s));
        PBNG_HIP(hipStreamSynchronize(s));
    } else {
        const int b = check_entries_host(pd);
        if (b >= 0) throw bad_entry(b);
        std::vector<i64> hrp(NU + 1);
        std::vector<i32> hci(M);
        for (int k = 0; k < ng; ++k) {
            const PackDesc &x = pd[k];
            for (i64 i = 0; i < x.n_u; ++i) hrp[x.u_off + i] = x.rp[i] + x.m_off;
            for (i64 j = 0; j < x.m; ++j) hci[x.m_off + j] = x.ci[j] + (i32)x.v_off;
        }
        hrp[NU] = M;
        PBNG_HIP(hipMemcpy(prp, hrp.data(), sizeof(i64) * (NU + 1), hipMemcpyHostToDevice));
        if (M) PBNG_HIP(hipMemcpy(pci, hci.data(), sizeof(i32) * M, hipMemcpyHostToDevice));
    }
    pbng_csr u{};
    u.n_u = NU;
    u.n_v = NV;
    u.m = M;
    u.row_ptr = prp;
    u.col_idx = pci;
    u.on_device = 1;
    DevGraph G;
    build_graph(c, u, G);
    const i64 nout = kind == 1 ? M : (side == 0 ? NU : NV);
    u64 *res = c.alloc<u64>(nout);
    if (kind == 1)
        wing_decompose(c, G, o, res);
    else
        tip_decompose(c, G, side, o, res);
    std::vector<OutDesc> od(ng);
    i64 off = 0;
    for (int k = 0; k < ng; ++k) {
        const pbng_csr &x = g[first + k];
        const i64 n = kind == 1 ? x.m : (side == 0 ? x.n_u : x.n_v);
        od[k] = OutDesc{outs[first + k], off, n};
        off += n;
    }
    if (on_dev) {
        OutDesc *dd = c.alloc<OutDesc>(ng);
        PBNG_HIP(hipMemcpy(dd, od.data(), sizeof(OutDesc) * ng, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_unpack, dim3(std::min(ng, 4096)), dim3(256), 0, s, (const OutDesc *)dd, ng, (const u64 *)res);
        PBNG_LAUNCH_CHECK();
    } else {
        for (int k = 0; k < ng; ++k)
            if (od[k].n)
                PBNG_HIP(hipMemcpyAsync(od[k].out, res + od[k].off, sizeof(u64) * od[k].n, hipMemcpyDeviceToHost, s));
    }
    PBNG_HIP(hipStreamSynchronize(s));
}

}  // namespace pbng
