// C ABI of the library (include/pbng.h): argument checks, host/device
// marshalling of the caller's graph, phase timing, error translation.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pbng_internal.h"

struct pbng_ctx {
    pbng::Ctx c;
};

// Work memory of pbng_count_noalloc: one array per device, held until the
// process ends.  Host code never uses its name as an address: pbng_create
// resolves the array's device address on the current device (once per
// device) and keeps it per device.
#define PBNG_SCRATCH_BYTES (size_t(64) << 20)
static __device__ __align__(256) unsigned char scratch[PBNG_SCRATCH_BYTES];

namespace pbng {

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on device dev (which must be current): looked
// up on the first call per device and kept.
hipError_t scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

struct CallScope {
    // Returns the arena to its free list when a call ends, however it ends.
    Ctx &c;
    explicit CallScope(Ctx &cc) : c(cc) { c.stats = pbng_stats{}; }
    ~CallScope() {
        (void)hipStreamSynchronize(c.stream);
        c.timing = false;
        c.arena.release_all();
    }
};

int fail(Ctx &c, int code, const std::string &msg) {
    c.last_error = msg;
    return code;
}

int check_csr(const pbng_csr *g) {
    if (!g) return PBNG_E_ARG;
    if (g->n_u < 0 || g->n_v < 0 || g->m < 0) return PBNG_E_ARG;
    if (!g->row_ptr) return PBNG_E_ARG;
    if (g->m > 0 && !g->col_idx) return PBNG_E_ARG;
    // label pair keys need n^2 < 2^64 and entry indices need 2m < 2^31
    if (g->n_u + g->n_v >= (int64_t(1) << 31) - 1) return PBNG_E_OVERFLOW;
    if (g->m >= (int64_t(1) << 30)) return PBNG_E_OVERFLOW;
    return 0;
}

// Device view of the caller's graph (copied in when it lives on the host).
pbng_csr device_graph(Ctx &c, const pbng_csr &g) {
    if (g.on_device) return g;
    pbng_csr d = g;
    i64 *rp = c.alloc<i64>(g.n_u + 1);
    i32 *ci = c.alloc<i32>(g.m);
    PBNG_HIP(hipMemcpyAsync(rp, g.row_ptr, sizeof(i64) * (g.n_u + 1), hipMemcpyHostToDevice, c.stream));
    if (g.m) PBNG_HIP(hipMemcpyAsync(ci, g.col_idx, sizeof(i32) * g.m, hipMemcpyHostToDevice, c.stream));
    d.row_ptr = rp;
    d.col_idx = ci;
    d.on_device = 1;
    return d;
}

// Output buffer on the device; copied back to the host when the caller's
// graph is on the host.
struct OutBuf {
    Ctx &c;
    u64 *user;
    u64 *dev;
    i64 n;
    bool host;
    OutBuf(Ctx &cc, u64 *u, i64 nn, bool h) : c(cc), user(u), dev(nullptr), n(nn), host(h) {
        dev = host ? c.alloc<u64>(n) : u;
    }
    void finish() {
        if (host && n) PBNG_HIP(hipMemcpyAsync(user, dev, sizeof(u64) * n, hipMemcpyDeviceToHost, c.stream));
        PBNG_HIP(hipStreamSynchronize(c.stream));
    }
};

pbng_opts default_opts(const pbng_opts *o) {
    pbng_opts d{};
    if (o) d = *o;
    return d;
}

// A NumPy .npy file holding exactly n little-endian float32 values in C
// order: magic, version, header length, a Python-literal header dict, data.
// Returns an empty string on success, else what is wrong.
std::string read_npy_f32(const char *path, i64 n, std::vector<float> &out) {
    FILE *f = fopen(path, "rb");
    if (!f) return "cannot open";
    struct Closer {
        FILE *f;
        ~Closer() { fclose(f); }
    } closer{f};
    unsigned char pre[10];
    if (fread(pre, 1, 8, f) != 8 || memcmp(pre, "\x93NUMPY", 6) != 0) return "not a .npy file";
    const int major = pre[6];
    size_t hlen = 0;
    if (major == 1) {
        if (fread(pre, 1, 2, f) != 2) return "truncated header";
        hlen = (size_t)pre[0] | ((size_t)pre[1] << 8);
    } else if (major == 2 || major == 3) {
        if (fread(pre, 1, 4, f) != 4) return "truncated header";
        hlen = (size_t)pre[0] | ((size_t)pre[1] << 8) | ((size_t)pre[2] << 16) | ((size_t)pre[3] << 24);
    } else {
        return "unknown .npy version";
    }
    if (hlen > (1u << 20)) return "header too long";
    std::string h(hlen, '\0');
    if (fread(&h[0], 1, hlen, f) != hlen) return "truncated header";
    auto compact = [](std::string t) {
        t.erase(std::remove_if(t.begin(), t.end(), [](char ch) { return ch == ' ' || ch == '\n'; }), t.end());
        return t;
    };
    const std::string hc = compact(h);
    if (hc.find("'descr':'<f4'") == std::string::npos) return "dtype is not little-endian float32";
    if (hc.find("'fortran_order':False") == std::string::npos) return "not in C order";
    const std::string shape = "'shape':(" + std::to_string(n) + ",)";
    if (hc.find(shape) == std::string::npos) return "shape is not (" + std::to_string(n) + ",)";
    out.resize((size_t)n);
    if (fread(out.data(), sizeof(float), (size_t)n, f) != (size_t)n) return "truncated data";
    return "";
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <class F>
int guarded(Ctx &c, F f) {
    try {
        f();
        return PBNG_OK;
    } catch (const Error &e) {
        return fail(c, e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(c, PBNG_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(c, PBNG_E_DEVICE, e.what());
    } catch (...) {
        return fail(c, PBNG_E_DEVICE, "unknown error");
    }
}

}  // namespace
}  // namespace pbng

using namespace pbng;

extern "C" {

int pbng_create(pbng_ctx **out, void *stream) {
    if (!out) return PBNG_E_ARG;
    *out = nullptr;
    pbng_ctx *x = nullptr;
    try {
        x = new pbng_ctx();
    } catch (...) {
        return PBNG_E_NOMEM;
    }
    x->c.stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&x->c.device) != hipSuccess) {
        delete x;
        return PBNG_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, x->c.device) == hipSuccess && prop.multiProcessorCount > 0)
        x->c.num_cu = prop.multiProcessorCount;
    if (scratch_address(x->c.device, &x->c.scratch) != hipSuccess) {
        (void)hipGetLastError();
        delete x;
        return PBNG_E_DEVICE;
    }
    // per-class work counters: every traversal kernel adds to them, so they
    // exist for the context's whole life
    if (hipMalloc(&x->c.kctr, sizeof(KCounters) * PBNG_K_NCLASS) != hipSuccess ||
        hipMemset(x->c.kctr, 0, sizeof(KCounters) * PBNG_K_NCLASS) != hipSuccess) {
        if (x->c.kctr) (void)hipFree(x->c.kctr);
        delete x;
        return PBNG_E_DEVICE;
    }
    *out = x;
    return PBNG_OK;
}

void pbng_destroy(pbng_ctx *x) {
    if (!x) return;
    (void)hipStreamSynchronize(x->c.stream);
    x->c.arena.destroy();
    if (x->c.sel_scratch) (void)hipFree(x->c.sel_scratch);
    if (x->c.kctr) (void)hipFree(x->c.kctr);
    if (x->c.mlp_p) (void)hipFree(x->c.mlp_p);
    if (x->c.cap_stream) (void)hipStreamDestroy(x->c.cap_stream);
    if (x->c.aux_stream) (void)hipStreamDestroy(x->c.aux_stream);
    for (hipEvent_t e : x->c.ev_pool) (void)hipEventDestroy(e);
    delete x;
}

const char *pbng_last_error(pbng_ctx *x) { return x ? x->c.last_error.c_str() : "null context"; }

int pbng_last_stats(pbng_ctx *x, pbng_stats *out) {
    if (!x || !out) return PBNG_E_ARG;
    *out = x->c.stats;
    return PBNG_OK;
}

int pbng_count(pbng_ctx *x, const pbng_csr *g, pbng_count_kind kind, const pbng_opts *opts, uint64_t *out) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (kind != PBNG_COUNT_VERTEX_U && kind != PBNG_COUNT_VERTEX_V && kind != PBNG_COUNT_EDGE)
        return fail(c, PBNG_E_ARG, "bad count kind");
    i64 nout = kind == PBNG_COUNT_VERTEX_U ? g->n_u : (kind == PBNG_COUNT_VERTEX_V ? g->n_v : g->m);
    if (nout > 0 && !out) return fail(c, PBNG_E_ARG, "null output");
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        pbng_csr dg = device_graph(c, *g);
        OutBuf ob(c, out, nout, !g->on_device);
        DevGraph G;
        build_graph(c, dg, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        auto t1 = std::chrono::steady_clock::now();
        if (kind == PBNG_COUNT_EDGE) {
            CountOut co;
            co.sup_edge = ob.dev;
            count_butterflies(c, G, co, o);
        } else {
            const u64 w = count_side(c, G, kind == PBNG_COUNT_VERTEX_U ? 0 : 1, o, ob.dev);
            c.stats.wedges_count += w;
            c.stats.wedges += w;
        }
        ob.finish();
        c.stats.ms_count = ms_since(t1);
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

int pbng_count_noalloc(pbng_ctx *x, const pbng_csr *g, pbng_count_kind kind, const pbng_opts *opts, uint64_t *out) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (!g->on_device) return fail(c, PBNG_E_ARG, "pbng_count_noalloc needs the graph and output in device memory");
    if (kind != PBNG_COUNT_VERTEX_U && kind != PBNG_COUNT_VERTEX_V && kind != PBNG_COUNT_EDGE)
        return fail(c, PBNG_E_ARG, "bad count kind");
    const i64 nout = kind == PBNG_COUNT_VERTEX_U ? g->n_u : (kind == PBNG_COUNT_VERTEX_V ? g->n_v : g->m);
    if (nout > 0 && !out) return fail(c, PBNG_E_ARG, "null output");
    // the vertex and edge arrays of the relabelled graph alone take 40 bytes
    // per edge and 32 per vertex; larger graphs are rejected before any work
    const i64 n = g->n_u + g->n_v;
    if ((u64)(40 * g->m + 32 * n) > PBNG_SCRATCH_BYTES)
        return fail(c, PBNG_E_OVERFLOW, "graph too large for the no-allocation scratch of " +
                                            std::to_string(PBNG_SCRATCH_BYTES >> 20) + " MiB");
    if (!c.scratch) return fail(c, PBNG_E_DEVICE, "no scratch address on this device");
    CallScope scope(c);
    // every block of this call comes from the scratch array (declared after
    // the call scope, so the fixed region is left before the arena's release)
    struct Fixed {
        Arena &a;
        Fixed(Arena &aa, void *base) : a(aa) {
            a.fixed_base = static_cast<char *>(base);
            a.fixed_cap = PBNG_SCRATCH_BYTES;
            a.fixed_used = 0;
        }
        ~Fixed() {
            a.fixed_base = nullptr;
            a.fixed_cap = a.fixed_used = 0;
        }
    } fixed(c.arena, c.scratch);
    pbng_opts o = default_opts(opts);
    o.flags &= ~PBNG_F_KERNEL_TIMING;  // timing events are created on demand
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call(false);
        DevGraph G;
        build_graph(c, *g, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        auto t1 = std::chrono::steady_clock::now();
        if (kind == PBNG_COUNT_EDGE) {
            CountOut co;
            co.sup_edge = out;
            count_butterflies(c, G, co, o);
        } else {
            const u64 w = count_side(c, G, kind == PBNG_COUNT_VERTEX_U ? 0 : 1, o, out);
            c.stats.wedges_count += w;
            c.stats.wedges += w;
        }
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_count = ms_since(t1);
        c.stats.ms_total = ms_since(t0);
    });
}

int pbng_tip(pbng_ctx *x, const pbng_csr *g, pbng_side side, const pbng_opts *opts, uint64_t *tip_out) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) return fail(c, PBNG_E_ARG, "bad side");
    i64 nout = side == PBNG_SIDE_U ? g->n_u : g->n_v;
    if (nout > 0 && !tip_out) return fail(c, PBNG_E_ARG, "null output");
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        pbng_csr dg = device_graph(c, *g);
        OutBuf ob(c, tip_out, nout, !g->on_device);
        DevGraph G;
        build_graph(c, dg, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        tip_decompose(c, G, side, o, ob.dev);
        ob.finish();
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

int pbng_tip_hinted(pbng_ctx *x, const pbng_csr *g, pbng_side side, const pbng_opts *opts, const uint64_t *theta_hint,
                    uint64_t *tip_out) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) return fail(c, PBNG_E_ARG, "bad side");
    const i64 nout = side == PBNG_SIDE_U ? g->n_u : g->n_v;
    if (nout > 0 && (!tip_out || !theta_hint)) return fail(c, PBNG_E_ARG, "null output or hint");
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    o.bound_rule = PBNG_BOUND_LEARNED;
    struct HintReset {
        Ctx &c;
        ~HintReset() { c.tip_hint = nullptr; }
    } reset{c};
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        pbng_csr dg = device_graph(c, *g);
        OutBuf ob(c, tip_out, nout, !g->on_device);
        u64 *hint = const_cast<u64 *>(theta_hint);
        if (!g->on_device && nout > 0) {
            hint = c.alloc<u64>(nout);
            PBNG_HIP(hipMemcpyAsync(hint, theta_hint, sizeof(u64) * nout, hipMemcpyHostToDevice, c.stream));
        }
        c.tip_hint = hint;
        DevGraph G;
        build_graph(c, dg, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        tip_decompose(c, G, side, o, ob.dev);
        ob.finish();
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

int pbng_tip_schedule(pbng_ctx *x, const pbng_csr *g, pbng_side side, const pbng_opts *opts, uint64_t *tip_out,
                      int32_t *part_out, uint64_t *init_out, uint64_t *bounds_out, int32_t bounds_cap, int32_t *nparts) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) return fail(c, PBNG_E_ARG, "bad side");
    const i64 nout = side == PBNG_SIDE_U ? g->n_u : g->n_v;
    if (nout > 0 && (!tip_out || !part_out || !init_out)) return fail(c, PBNG_E_ARG, "null output");
    if (bounds_cap < 0 || (bounds_cap > 0 && !bounds_out) || !nparts) return fail(c, PBNG_E_ARG, "bad bounds output");
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    struct SchedReset {
        Ctx &c;
        ~SchedReset() {
            c.sched_part = nullptr;
            c.sched_init = nullptr;
            c.sched_bounds = nullptr;
            c.sched_cap = 0;
        }
    } reset{c};
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        const bool host = !g->on_device;
        pbng_csr dg = device_graph(c, *g);
        OutBuf ob(c, tip_out, nout, host);
        c.sched_part = host ? c.alloc<i32>(nout) : part_out;
        c.sched_init = host ? c.alloc<u64>(nout) : init_out;
        c.sched_bounds = host ? c.alloc<u64>(bounds_cap) : bounds_out;
        c.sched_cap = bounds_cap;
        c.sched_np = 0;
        DevGraph G;
        build_graph(c, dg, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        if (nout > 0) tip_decompose(c, G, side, o, ob.dev);
        if (host && nout > 0) {
            PBNG_HIP(hipMemcpyAsync(part_out, c.sched_part, sizeof(i32) * nout, hipMemcpyDeviceToHost, c.stream));
            PBNG_HIP(hipMemcpyAsync(init_out, c.sched_init, sizeof(u64) * nout, hipMemcpyDeviceToHost, c.stream));
            const i32 nb = std::min<i32>(c.sched_np, bounds_cap);
            if (nb > 0)
                PBNG_HIP(hipMemcpyAsync(bounds_out, c.sched_bounds, sizeof(u64) * nb, hipMemcpyDeviceToHost, c.stream));
        }
        ob.finish();
        *nparts = c.sched_np;
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

namespace pbng {
namespace {
int components_call(pbng_ctx *x, const pbng_csr *g, int what, const uint64_t *theta, uint64_t k, int32_t *comp) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    const i64 n = what == 2 ? g->m : (what == 0 ? g->n_u : g->n_v);
    if (n > 0 && (!theta || !comp)) return fail(c, PBNG_E_ARG, "null entity numbers or output");
    CallScope scope(c);
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call(false);
        const bool host = !g->on_device;
        pbng_csr dg = device_graph(c, *g);
        const u64 *th = theta;
        i32 *out = comp;
        if (host && n > 0) {
            u64 *t = c.alloc<u64>(n);
            PBNG_HIP(hipMemcpyAsync(t, theta, sizeof(u64) * n, hipMemcpyHostToDevice, c.stream));
            th = t;
            out = c.alloc<i32>(n);
        }
        DevGraph G;
        build_graph(c, dg, G);
        level_components(c, G, what, th, k, out);
        if (host && n > 0) PBNG_HIP(hipMemcpyAsync(comp, out, sizeof(i32) * n, hipMemcpyDeviceToHost, c.stream));
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_total = ms_since(t0);
    });
}
}  // namespace
}  // namespace pbng

int pbng_tip_components(pbng_ctx *x, const pbng_csr *g, pbng_side side, const uint64_t *theta, uint64_t k,
                        int32_t *comp_out) {
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) {
        if (x) x->c.last_error = "bad side";
        return PBNG_E_ARG;
    }
    return components_call(x, g, side == PBNG_SIDE_U ? 0 : 1, theta, k, comp_out);
}

int pbng_wing_components(pbng_ctx *x, const pbng_csr *g, const uint64_t *theta, uint64_t k, int32_t *comp_out) {
    return components_call(x, g, 2, theta, k, comp_out);
}

int pbng_wing(pbng_ctx *x, const pbng_csr *g, const pbng_opts *opts, uint64_t *wing_out) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (g->m > 0 && !wing_out) return fail(c, PBNG_E_ARG, "null output");
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        pbng_csr dg = device_graph(c, *g);
        OutBuf ob(c, wing_out, g->m, !g->on_device);
        DevGraph G;
        build_graph(c, dg, G);
        PBNG_HIP(hipStreamSynchronize(c.stream));
        c.stats.ms_prep = ms_since(t0);
        wing_decompose(c, G, o, ob.dev);
        ob.finish();
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

}  // extern "C"

namespace pbng {
namespace {

void add_stats(pbng_stats &a, const pbng_stats &b) {
    a.ms_prep += b.ms_prep;
    a.ms_count += b.ms_count;
    a.ms_cd += b.ms_cd;
    a.ms_fd_prep += b.ms_fd_prep;
    a.ms_fd += b.ms_fd;
    a.wedges += b.wedges;
    a.wedges_count += b.wedges_count;
    a.wedges_cd += b.wedges_cd;
    a.wedges_fd += b.wedges_fd;
    a.updates += b.updates;
    a.links += b.links;
    a.blooms += b.blooms;
    a.bloom_pairs += b.bloom_pairs;
    a.rho += b.rho;
    a.recounts += b.recounts;
    a.partitions += b.partitions;
    a.P_used = b.P_used;
    a.bound_rule_used = b.bound_rule_used;
    a.fd_work_max = std::max(a.fd_work_max, b.fd_work_max);
    a.fd_work_sum += b.fd_work_sum;
    a.dense_pairs += b.dense_pairs;
    a.fd_wide += b.fd_wide;
}

int batch_call(pbng_ctx *x, const pbng_csr *g, int32_t ng, int kind, int side, const pbng_opts *opts,
               uint64_t *const *outs) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    if (ng < 0 || (ng > 0 && (!g || !outs))) return fail(c, PBNG_E_ARG, "bad batch arguments");
    for (int k = 0; k < ng; ++k) {
        const int rc = check_csr(&g[k]);
        if (rc) return fail(c, rc, "bad graph arguments in batch entry " + std::to_string(k));
        if ((g[k].on_device != 0) != (g[0].on_device != 0))
            return fail(c, PBNG_E_ARG, "batch mixes host and device graphs");
        const i64 n = kind == 1 ? g[k].m : (side == 0 ? g[k].n_u : g[k].n_v);
        if (n > 0 && !outs[k]) return fail(c, PBNG_E_ARG, "null output in batch entry " + std::to_string(k));
    }
    CallScope scope(c);
    pbng_opts o = default_opts(opts);
    // per-workgroup scratch of the largest starts and of spilled hash keys
    // scales with the union's vertex count, so unions stay moderate
    const i64 max_m = o.batch_edges > 0 ? (i64)o.batch_edges : (i64(1) << 26);
    return guarded(c, [&] {
        auto t0 = std::chrono::steady_clock::now();
        c.timing_begin_call((o.flags & PBNG_F_KERNEL_TIMING) != 0);
        pbng_stats acc{};
        for (int first = 0; first < ng;) {
            const int last = (int)batch_chunk_end(g, ng, first, max_m);
            c.stats = pbng_stats{};
            batch_run(c, g, first, last, kind, side, o, outs);
            add_stats(acc, c.stats);
            c.arena.release_all();
            first = last;
        }
        c.stats = acc;
        if (o.flags & PBNG_F_KERNEL_TIMING) c.timing_end_call();
        c.stats.ms_total = ms_since(t0);
    });
}

}  // namespace
}  // namespace pbng

extern "C" {

int pbng_tip_batch(pbng_ctx *x, const pbng_csr *g, int32_t ng, pbng_side side, const pbng_opts *opts,
                   uint64_t *const *outs) {
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) {
        if (x) x->c.last_error = "bad side";
        return PBNG_E_ARG;
    }
    return batch_call(x, g, ng, 0, side, opts, outs);
}

int pbng_wing_batch(pbng_ctx *x, const pbng_csr *g, int32_t ng, const pbng_opts *opts, uint64_t *const *outs) {
    return batch_call(x, g, ng, 1, 0, opts, outs);
}

int pbng_autotune(pbng_ctx *x, const pbng_csr *g, int32_t kind, const pbng_opts *base, pbng_opts *best,
                  double *ms_best) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (kind < 0 || kind > 2 || !best) return fail(c, PBNG_E_ARG, "bad autotune arguments");
    CallScope scope(c);
    return guarded(c, [&] {
        c.timing_begin_call(false);
        pbng_csr dg = device_graph(c, *g);
        DevGraph G;
        build_graph(c, dg, G);
        const std::array<i64, 5> key{g->n_u, g->n_v, g->m, G.maxdeg, (i64)kind};
        auto hit = c.tune_cache.find(key);
        if (hit != c.tune_cache.end()) {
            *best = hit->second.first;
            if (ms_best) *ms_best = hit->second.second;
            return;
        }
        const i64 nout = kind == 2 ? g->m : (kind == 0 ? g->n_u : g->n_v);
        u64 *out = c.alloc<u64>(nout);
        const size_t mk = c.arena.mark();
        auto run = [&](const pbng_opts &o) {
            c.stats = pbng_stats{};
            auto t0 = std::chrono::steady_clock::now();
            if (kind == 2)
                wing_decompose(c, G, o, out);
            else
                tip_decompose(c, G, kind, o, out);
            PBNG_HIP(hipStreamSynchronize(c.stream));
            const double ms = ms_since(t0);
            c.arena.release_to(mk);
            return ms;
        };
        pbng_opts cur = default_opts(base);
        cur.flags &= ~PBNG_F_KERNEL_TIMING;
        run(cur);
        double best_ms = run(cur);
        auto try_knob = [&](int32_t pbng_opts::*field, std::initializer_list<int32_t> values) {
            const int32_t keep = cur.*field;
            int32_t win = keep;
            for (int32_t v : values) {
                if (v == keep) continue;
                cur.*field = v;
                const double ms = run(cur);
                if (ms < best_ms) {
                    best_ms = ms;
                    win = v;
                }
            }
            cur.*field = win;
        };
        // tip: the paper's range rule against the library's plain rule (a
        // caller's learned or random rule is kept)
        if (kind != 2 && (cur.bound_rule == PBNG_BOUND_PLAIN || cur.bound_rule == PBNG_BOUND_PAPER))
            try_knob(&pbng_opts::bound_rule, {PBNG_BOUND_PLAIN, PBNG_BOUND_PAPER});
        try_knob(&pbng_opts::dense_cut, {-1, 256, 1024, 4096});
        if (kind != 2) {
            try_knob(&pbng_opts::tile_w, {1 << 16, 1 << 18, 1 << 20, -1});
            // the Section 5.1 recount bound against never recounting
            try_knob(&pbng_opts::recount_w, {0, -1});
        } else {
            // wing: fine-grained work above which a partition is peeled
            // device-wide
            try_knob(&pbng_opts::wide_work, {1 << 22, 1 << 26, -1});
        }
        const int32_t p0 = cur.P > 0 ? cur.P : (kind == 2 ? 400 : 150);
        try_knob(&pbng_opts::P, {std::max(1, p0 / 2), p0 * 2});
        *best = cur;
        if (ms_best) *ms_best = best_ms;
        c.tune_cache[key] = {cur, best_ms};
    });
}

int pbng_tip_features(pbng_ctx *x, const pbng_csr *g, pbng_side side, float *feat) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    int rc = check_csr(g);
    if (rc) return fail(c, rc, "bad graph arguments");
    if (side != PBNG_SIDE_U && side != PBNG_SIDE_V) return fail(c, PBNG_E_ARG, "bad side");
    const i64 nx = side == PBNG_SIDE_U ? g->n_u : g->n_v;
    if (nx > 0 && !feat) return fail(c, PBNG_E_ARG, "null output");
    CallScope scope(c);
    return guarded(c, [&] {
        c.timing_begin_call(false);
        pbng_csr dg = device_graph(c, *g);
        DevGraph G;
        build_graph(c, dg, G);
        u64 *sup = c.alloc<u64>(nx);
        count_side(c, G, side, pbng_opts{}, sup);
        float *F = g->on_device ? feat : c.alloc<float>(nx * 8);
        tip_features(c, G, side, sup, F);
        if (!g->on_device && nx)
            PBNG_HIP(hipMemcpyAsync(feat, F, sizeof(float) * nx * 8, hipMemcpyDeviceToHost, c.stream));
        PBNG_HIP(hipStreamSynchronize(c.stream));
    });
}

int pbng_predictor_load(pbng_ctx *x, const char *path) {
    if (!x) return PBNG_E_ARG;
    Ctx &c = x->c;
    if (!path) return fail(c, PBNG_E_ARG, "null path");
    std::vector<float> p;
    const std::string err = read_npy_f32(path, PBNG_MLP_NPARAM, p);
    if (!err.empty()) return fail(c, PBNG_E_ARG, std::string(path) + ": " + err);
    return guarded(c, [&] { mlp_set(c, p.data()); });
}

int pbng_mlp_init(pbng_ctx *x, uint64_t seed) {
    if (!x) return PBNG_E_ARG;
    return guarded(x->c, [&] { mlp_init(x->c, seed); });
}

int pbng_mlp_set(pbng_ctx *x, const float *params) {
    if (!x || !params) return PBNG_E_ARG;
    return guarded(x->c, [&] { mlp_set(x->c, params); });
}

int pbng_mlp_get(pbng_ctx *x, float *params) {
    if (!x || !params) return PBNG_E_ARG;
    return guarded(x->c, [&] { mlp_get(x->c, params); });
}

int pbng_mlp_forward(pbng_ctx *x, const float *in, int64_t n, float *out) {
    if (!x || n < 0 || (n > 0 && (!in || !out))) return PBNG_E_ARG;
    Ctx &c = x->c;
    return guarded(c, [&] {
        mlp_forward(c, in, n, out);
        PBNG_HIP(hipStreamSynchronize(c.stream));
    });
}

int pbng_mlp_loss_grad(pbng_ctx *x, const float *in, const float *r, const float *wt, int64_t n, float *grad,
                       float *loss) {
    if (!x || n < 0 || !grad || !loss || (n > 0 && (!in || !r || !wt))) return PBNG_E_ARG;
    Ctx &c = x->c;
    CallScope scope(c);
    return guarded(c, [&] { mlp_loss_grad(c, in, r, wt, n, grad, loss); });
}

int pbng_mlp_train(pbng_ctx *x, const float *in, const float *r, const float *wt, int64_t n, int32_t batch,
                   int32_t epochs, float lr, float *epoch_loss) {
    if (!x || n < 0 || batch <= 0 || epochs < 0 || (n > 0 && (!in || !r || !wt))) return PBNG_E_ARG;
    Ctx &c = x->c;
    CallScope scope(c);
    return guarded(c, [&] { mlp_train(c, in, r, wt, n, batch, epochs, lr, epoch_loss); });
}

}  // extern "C"
