// Internal declarations of the gfx950 butterfly-peeling library.
// Host orchestration is C++17 over the HIP runtime; kernels are HIP for
// CDNA4 (wave64).  Nothing here is exported: the C ABI is in include/pbng.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pbng.h"

namespace pbng {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef int32_t i32;

constexpr int WAVE = 64;

// Error carried to the C ABI boundary, where it becomes a return code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PBNG_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            throw ::pbng::Error(e_ == hipErrorOutOfMemory ? PBNG_E_NOMEM : PBNG_E_DEVICE, \
                                std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PBNG_LAUNCH_CHECK() PBNG_HIP(hipGetLastError())

// Device memory cache owned by a context: blocks are reused across calls and
// freed by pbng_destroy.  take() returns a block of at least `bytes`.
struct Arena {
    std::multimap<size_t, void *> free_blocks;
    std::vector<std::pair<void *, size_t>> in_use;
    size_t bytes_held = 0;
    // Fixed region: while fixed_base is set, take() carves blocks out of
    // [fixed_base, fixed_base + fixed_cap) by bumping fixed_used, never
    // allocates, and throws PBNG_E_NOMEM once the region is exhausted.
    char *fixed_base = nullptr;
    size_t fixed_cap = 0, fixed_used = 0;
    void *take(size_t bytes);
    void release_all();  // back to the free list (end of a call)
    size_t mark() const { return fixed_base ? fixed_used : in_use.size(); }
    void release_to(size_t mark);  // blocks taken after `mark` back to the free list
    size_t fixed_left() const { return fixed_base ? fixed_cap - fixed_used : ~size_t(0); }
    void destroy();      // hipFree everything
};

// Algorithmic-work counters a traversal kernel adds to (one set per kernel
// class): wedges walked, list segments opened, 64-bit atomic updates.
struct KCounters {
    u64 wedges, segments, atomics, items;
};

struct Ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 256;
    Arena arena;
    std::string last_error;
    pbng_stats stats{};
    // device scratch of the range selection, kept for the context's life
    void *sel_scratch = nullptr;
    // kernel-class timing (PBNG_F_KERNEL_TIMING)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> intervals[PBNG_K_NCLASS];
    KCounters *kctr = nullptr;  // device [PBNG_K_NCLASS], zeroed per call
    // learned range-bound predictor: parameters, Adam moments, gradient sums
    float *mlp_p = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_g = nullptr, *mlp_acc = nullptr;
    int mlp_t = 0;
    bool mlp_ready = false;
    // autotuner: best settings and their time per graph signature
    std::map<std::array<i64, 5>, std::pair<pbng_opts, double>> tune_cache;
    // stream used only to capture round graphs (replayed on `stream`)
    hipStream_t cap_stream = nullptr;
    hipStream_t capture_stream();
    // predicted tip numbers supplied for one call (pbng_tip_hinted, device)
    const u64 *tip_hint = nullptr;
    // device address of the library's static scratch array on this
    // context's device (pbng_count_noalloc)
    void *scratch = nullptr;
    // schedule outputs of a tip call (device pointers, set by
    // pbng_tip_schedule for one call): partition of each vertex, support at
    // its partition's start, exclusive upper bound of each partition
    i32 *sched_part = nullptr;
    u64 *sched_init = nullptr;
    u64 *sched_bounds = nullptr;
    i32 sched_cap = 0;
    i32 sched_np = 0;
    // second stream for work that overlaps the context stream's
    hipStream_t aux_stream = nullptr;
    hipStream_t aux();
    template <class T>
    T *alloc(size_t n) {
        return static_cast<T *>(arena.take((n ? n : 1) * sizeof(T)));
    }
    hipEvent_t event();
    // interval of kernel class cls on stream st (the context stream if null)
    void kbegin(int cls, hipStream_t st = nullptr);
    void kend(int cls, hipStream_t st = nullptr);
    void timing_begin_call(bool on);
    void timing_end_call();  // fills stats.kstat (synchronises)

};

// Graph in device memory after preprocessing (Algorithm 1, priority
// assignment and sorted adjacency).  Global vertex ids: U = [0, n_u),
// V = [n_u, n_u + n_v).  A label is the vertex's position in the order of
// decreasing degree (ties by increasing global id).
struct DevGraph {
    i64 n_u = 0, n_v = 0, n = 0, m = 0;
    i64 maxdeg = 0;
    const i64 *urow = nullptr;  // U-side CSR (caller's, on device)
    const i32 *ucol = nullptr;
    i64 *vrow = nullptr;        // V-side CSR: U ids, and edge ids
    i32 *vadj = nullptr;
    i32 *veid = nullptr;
    i32 *label = nullptr;       // [n] global id -> label
    i32 *gid = nullptr;         // [n] label -> global id
    i64 *loff = nullptr;        // [n+1] label CSR offsets
    i32 *ladj = nullptr;        // [2m] neighbour labels, ascending per row
    i32 *leid = nullptr;        // [2m] edge id of each entry
    i32 *lpl = nullptr;         // [2m] wedge-prefix length of (row, entry), see prep
    i64 *wsum = nullptr;        // [n+1] exclusive prefix of lpl per row (wedges per start)
};

// ---- primitives (prims.hip) ----
template <class T>
void exclusive_scan(Ctx &c, const T *in, T *out, i64 n);  // out[0..n], out[n] = total
void radix_sort_u64(Ctx &c, u64 *keys, i32 *vals, i64 n, int bits, u64 **keys_out, i32 **vals_out);
void iota_i32(Ctx &c, i32 *p, i64 n);
template <class T>
void fill(Ctx &c, T *p, T v, i64 n);
u64 reduce_sum_u64(Ctx &c, const u64 *p, i64 n);  // synchronous
template <class T>
T read_scalar(Ctx &c, const T *dev);               // synchronous

// ---- graph preprocessing (prep.hip) ----
void build_graph(Ctx &c, const pbng_csr &g, DevGraph &G);

// ---- counting (count.hip) ----
struct CountOut {
    u64 *sup_label = nullptr;  // [n] per-vertex butterflies by label (or null)
    u64 *sup_edge = nullptr;   // [m] per-edge butterflies (or null)
};
void count_butterflies(Ctx &c, const DevGraph &G, const CountOut &out, const pbng_opts &o);
// Per-vertex counts of the rows of an arbitrary "peeled side" view are
// produced by count_butterflies on the full graph and gathered by label.
void gather_side(Ctx &c, const DevGraph &G, const u64 *sup_label, int side, u64 *out);

// BE-Index (Section 2.3) built from the counting traversal.
struct BEIndex {
    i64 nblooms = 0, npairs = 0;
    i64 *boff = nullptr;   // [nblooms+1] pair offsets per bloom
    u32 *bk = nullptr;     // [nblooms] live pairs (bloom number k_B)
    i32 *bedge = nullptr;  // [2*npairs] edge ids, pair p at 2p, 2p+1 (twins)
    i64 *eoff = nullptr;   // [m+1] link offsets per edge
    i32 *ebloom = nullptr; // [2*npairs] bloom of each link
    i32 *etwin = nullptr;  // [2*npairs] twin edge of each link
    i32 *pbloom = nullptr; // [npairs] bloom of each pair
};
void build_be_index(Ctx &c, const DevGraph &G, BEIndex &I, u64 *sup_edge);

// ---- decompositions ----
void tip_decompose(Ctx &c, const DevGraph &G, int side, const pbng_opts &o, u64 *theta_dev);
void wing_decompose(Ctx &c, const DevGraph &G, const pbng_opts &o, u64 *theta_dev);
// k-tips (what 0: side U, 1: side V) or k-wings (what 2) from entity numbers
// theta: comp[i] = smallest id of entity i's component at level k, or -1
void level_components(Ctx &c, const DevGraph &G, int what, const u64 *theta, u64 k, i32 *comp);

// ---- range selection (select.hip) ----
// Smallest s with sum{w_l : active_l, key_l <= s} >= target; if the total is
// below target, the largest active key.  Result written to *s_out (device).
// The target is *target_dev, or, when scale_dev is given, the plain rule's
// scale * (alive work) / parts_left computed on the device.  A nonzero
// count_target also ends the range where #{active_l : key_l <= s} reaches it
// (s is the smaller of the two crossings).
void weighted_select(Ctx &c, const u64 *key, const u64 *w, const unsigned char *state,
                     unsigned char alive_code, i64 n, const u64 *target_dev, const double *scale_dev,
                     int parts_left, u64 *s_out, u64 *work_at_s_out, u64 count_target = 0);

// Counting pass with an optional alive filter by label (recounts).
// Returns the wedges walked.  sup_label / sup_edge are overwritten.
u64 count_pass(Ctx &c, const DevGraph &G, u64 *sup_label, u64 *sup_edge, const unsigned char *alive_label);

// One-side counting without hub-hub butterflies (lclass by label: 0 other
// side, 1 this side, 2 hub of this side); see count.hip.
u64 count_pass_xside(Ctx &c, const DevGraph &G, u64 *sup_label, const unsigned char *lclass);

// Per-vertex butterfly counts of one side (0 = U, 1 = V) into out[n_side]:
// hub-hub butterflies of that side from an int8 Gram matrix on matrix cores
// when the options allow it (mfma.hip), everything else by traversal.
// Returns the wedges walked.
u64 count_side(Ctx &c, const DevGraph &G, int side, const pbng_opts &o, u64 *out);

// owner of an instantiated HIP graph
struct GraphExec {
    hipGraphExec_t e = nullptr;
    GraphExec() = default;
    GraphExec(const GraphExec &) = delete;
    GraphExec &operator=(const GraphExec &) = delete;
    ~GraphExec() {
        if (e) (void)hipGraphExecDestroy(e);
    }
};

// Work forked onto the context's second stream and joined back: fork()
// makes the second stream wait for everything queued so far on the context
// stream; join() makes the context stream wait for the second stream.
struct StreamJoin {
    Ctx &c;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool forked = false;
    explicit StreamJoin(Ctx &cc) : c(cc) {}
    StreamJoin(const StreamJoin &) = delete;
    StreamJoin &operator=(const StreamJoin &) = delete;
    void fork() {
        aux = c.aux();
        PBNG_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        PBNG_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        PBNG_HIP(hipEventRecord(ev_fork, c.stream));
        PBNG_HIP(hipStreamWaitEvent(aux, ev_fork, 0));
        forked = true;
    }
    void join() {
        if (!forked) return;
        PBNG_HIP(hipEventRecord(ev_join, aux));
        PBNG_HIP(hipStreamWaitEvent(c.stream, ev_join, 0));
        forked = false;
    }
    ~StreamJoin() {
        if (aux) (void)hipStreamSynchronize(aux);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }
};

// many graphs per call (batch.hip)
i64 batch_chunk_end(const pbng_csr *g, int ng, int first, i64 max_m);
void batch_run(Ctx &c, const pbng_csr *g, int first, int last, int kind, int side, const pbng_opts &o,
               uint64_t *const *outs);

// learned range bounds (learned.hip)
void mlp_init(Ctx &c, u64 seed);
void mlp_set(Ctx &c, const float *host);
void mlp_get(Ctx &c, float *host);
void mlp_forward(Ctx &c, const float *X, i64 n, float *out);
void mlp_loss_grad(Ctx &c, const float *X, const float *Y, const float *Wt, i64 n, float *grad, float *loss_host);
void mlp_train(Ctx &c, const float *X, const float *Y, const float *Wt, i64 n, int batch, int epochs, float lr,
               float *epoch_loss);
void tip_features(Ctx &c, const DevGraph &G, int side, const u64 *sup, float *F);
void learned_theta_hat(Ctx &c, const DevGraph &G, int side, const u64 *sup, u64 *theta_hat);

// histograms over small key ranges (out += counts / sums of val per key)
void hist_add_u32(Ctx &c, const i32 *key, i64 n, i32 nb, u32 *out);
void hist_add_u64(Ctx &c, const i32 *key, const u64 *val, i64 n, i32 nb, u64 *out);

int bits_for(u64 maxval);
int grid_1d(i64 n, int block = 256, int cap = 16384);

}  // namespace pbng
