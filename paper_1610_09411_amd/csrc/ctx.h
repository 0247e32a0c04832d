// Host-side context shared by the pipeline stages.  All device memory is
// owned here: buffers grow on demand and are reused across calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <stdio.h>
#include <vector>
#include <initializer_list>
#include "escape.h"

// Indices of the exact 128-bit sums produced on the device.  Each stage adds
// its terms into acc[2*slot] (lo) / acc[2*slot+1] (hi).
enum AccSlot {
    AC_W,      // sum_v C(d,2)                      wedges
    AC_S3,     // sum_v C(d,3)                      3-stars
    AC_S4,     // sum_v C(d,4)                      4-stars (pattern 1)
    AC_T3,     // sum_e t(e) = 3 T
    AC_TT,     // sum_v t(v)(d(v)-2)                tailed triangles
    AC_D,      // sum_e C(t(e),2)                   diamonds
    AC_C4,     // 4-cycles
    AC_K4X4,   // sum_t K4(t) = 4 K4
    AC_EP,     // sum_e (d(u)-1)(d(v)-1)
    AC_N2,     // sum over ordered edges (d(j)-1) C(d(i)-1,2)
    AC_N3,     // sum_i sum_{j<k in N(i)} (d(j)-1)(d(k)-1)
    AC_N4,     // sum_i t(i) C(d(i)-2,2)
    AC_N5,     // sum over ordered edges (d(i)-1)(t(j)-t(ij))
    AC_N6,     // sum_e t(e)(d(u)-2)(d(v)-2)
    AC_N7X2,   // sum_e C4(e)(d(u)+d(v)-4) = 2 sum_v C4(v)(d(v)-2)
    AC_N9,     // sum_v C(t(v),2)
    AC_N10,    // sum_t sum_{k in t} (t(opposite edge)-1)(d(k)-2)
    AC_N11,    // sum over ordered edges C(t(e),2)(d(i)-3)
    AC_N12,    // sum_e C4(e) t(e)
    AC_N13,    // sum over pairs C(W(i,j),3)
    AC_N14,    // sum_e C(t(e),3)
    AC_N15,    // sum_v K4(v)(d(v)-3)
    AC_N16,    // sum_t sum_{i in t} (t(ij)-1)(t(ik)-1)
    AC_N17,    // sum over pairs (W(i,j)-2) D(i,j)
    AC_N18,    // wheels
    AC_N19,    // sum_e K4(e)(t(e)-2)
    AC_N20,    // sum_t C(K4(t),2)
    AC_CYC,    // sum over ordered pairs P(i,j) Wnt(i,j)
    AC_Z,      // directed tailed triangles of the 5-cycle correction
    AC_K5,     // 5-cliques
    AC_SW,     // sum_b [C(d_b,2) d_b + (d_b-1) sum_{a in N(b)} d_a]
    AC_TD,     // sum_v t(v) d(v)
    AC_WD2,    // wheels of the dense hubs, twice over: sum over rim pairs of C(c,2)
    AC_COUNT
};

enum Buf {
    B_RP_IN, B_COL_IN,          // input CSR copied to the device
    B_DEG, B_PERM, B_RANK,      // degree (input ids), rank -> input id, input id -> rank
    B_KEYS_A, B_KEYS_B, B_VALS_A, B_VALS_B, B_HIST,
    B_OFF, B_ADJ, B_SPLIT,      // relabelled CSR (rank ids), rows sorted
    B_EOFF, B_ARC_EID, B_REV,   // out-arc prefix, edge id of each arc, reverse arc
    B_EARC, B_ELO,              // out-arc position and lower endpoint of each edge
    B_TE, B_TV, B_K4E, B_C4E,   // per-edge / per-vertex fragment counts
    B_TARC,                     // t(e) of each arc's edge, indexed like adj
    B_AOFF, B_ACUR, B_AA, B_AV, // per-arc triangle lists: offsets, cursors, arc index of apex, apex id
    B_SEGCLS, B_SEGQ,           // segmented-sort work lists
    B_SCAN_TMP,
    B_ACC, B_ERR, B_OUT, B_WORK,
    B_WG_SCRATCH,               // per-workgroup dense tables for the pair passes
    B_WG_TOUCH,
    B_TASK,
    B_FRAG,                     // fragment outputs in input order
    B_OB, B_OB_OFF,             // out-neighbourhood bitmaps for 5-cliques
    B_K5_UNITS,                 // offsets of the 5-clique work units per vertex
    B_CAN_CNT, B_CAN_LEN, B_CAN_OFF, B_CAN_UOFF, B_CAN_ARCS,   // canonicalisation work
    B_CAN_RP, B_CAN_COL,        // canonical CSR
    B_GOFF,                     // batched: vertex and arc offsets of the graphs (int64, 2 x (G+1))
    B_VGRAPH,                   // batched: graph of each union vertex id (= of each rank)
    B_URP, B_UCOL,              // batched: CSR of the disjoint union
    B_BOUT,                     // batched: per-graph counts and overflow flags
    B_TASK_OWNER,               // vertex of each task of a split per-vertex pass
    B_TRIREC,                   // triangles found by the count pass: 3 arcs and 3 slots each
    B_TRICNT,                   // count of B_TRIREC entries, bound of oriented wedges
    B_K5_DENSE,                 // vertices whose 5-cliques are counted through the complement
    B_K5_DENSE_SCR,             // per-workgroup complement rows of those vertices
    B_HUB_DID,                  // pattern 17 hub pairs: number of each dense arc (or -1)
    B_HUB_CNT, B_HUB_BASE,      // dense arcs per row and their exclusive prefix
    B_HUB_KR,                   // first and last row of each chunk of dense edges
    B_HUB_W,                    // W(i,j) of the hub pairs, R x R
    B_HUB_Y,                    // one chunk of the hub / dense-edge incidence bytes
    B_WD_S2, B_WD_FLAG,         // wheels of dense hubs: sum of t^2 per candidate, chosen flags
    B_WD_Y, B_WD_META,          // their adjacency matrices (a batch of hubs) and batch tables
    B_K4_LIST, B_K4_CNT, B_K4_FLAG,   // 4-cliques of dense rows: candidates, count, chosen flags
    B_K4_Y, B_K4_META,          // their B_a and C_a matrices (a batch) and batch tables
    B_TRIBIG,                   // triangles: vertices whose N+ takes a workgroup's hash set
    B_COUNT
};

#define NSTAGES 10
// stage numbers (esc_last_profile order) of the stages with products
#define STAGE_K4 3
#define STAGE_PAIRS 6
#define STAGE_WHEELS 7

// Per-graph sums: graph g's slots start at acc + g * ACC_STRIDE.
#define ACC_STRIDE (2 * AC_COUNT)

// Which graph an item of the union belongs to: vg maps a rank (equivalently
// a union vertex id) to its graph, voff holds the first rank of every graph.
// A single-graph call passes vg = nullptr: graph 0 spans [0, n).
struct GMap {
    const int32_t *vg;
    const int64_t *voff;
    int32_t n;
    __device__ int graph(int32_t r) const { return vg ? vg[r] : 0; }
    __device__ int32_t begin(int g) const { return vg ? (int32_t)voff[g] : 0; }
    __device__ int32_t end(int g) const { return vg ? (int32_t)voff[g + 1] : n; }
};

struct esc_ctx;
inline int pair_wgs(const esc_ctx *c);

#define TUNE_SLOTS 64   // entries of a context's tuning table

struct esc_ctx {
    int device;
    size_t budget;
    hipStream_t own_stream;
    hipStream_t stream;        // stream of the current call
    void *buf[B_COUNT];
    size_t cap[B_COUNT];
    size_t held;
    int num_cu;
    int max_lds;               // bytes of LDS one workgroup may allocate
    uint64_t work[ESC_WORK_COUNTERS];
    float stage_ms[NSTAGES];
    // stages with a matrix-core product after their walk: an event at the
    // walk's end (walk_rec), the walk's and the product's times and the
    // product's multiply-adds (see esc_last_products)
    hipEvent_t ev_walk[NSTAGES];
    bool walk_rec[NSTAGES];
    float walk_ms[NSTAGES], prod_ms[NSTAGES];
    uint64_t prod_macs[NSTAGES];
    uint64_t visits[NSTAGES];
    esc_u128 noninduced[45];
    esc_u128 three[4];         // induced 3-vertex counts of the last single-graph call
    hipEvent_t ev[NSTAGES + 1];
    // current graph
    int32_t n;
    int64_t m2;                // number of arcs (2m)
    int64_t m;
    int64_t narcs_apex;        // total per-arc triangle list entries (6T)
    int32_t maxdeg;
    int32_t maxdplus;
    uint64_t key_w, key_dp;    // W and the directed 3-path bound of the call, after the degree order
    int k;
    uint32_t flags;
    bool scratch_clean;        // per-workgroup tables are all zero
    // batched calls: the graphs form one disjoint union whose rank order is
    // (graph, degree, id), so every graph owns a contiguous range of ranks
    int32_t G;                 // number of graphs; 0 for a single-graph call
    int32_t tab_n;             // extent of a per-workgroup dense table (largest graph)
    int task_chunk;            // sources taken per grab by the per-source kernels
    int32_t *d_inv4, *d_inv5;  // signed inverse matrices (Appendix B), device copies
    const int32_t *av;         // apex ids of the triangle lists, or nullptr (read through aa)
    int wg_per_cu;             // workgroups per CU of the per-source kernels
    int wg_cap;                // largest wg_per_cu the tables' memory allows for this call
    int k5_work_log2;          // 5-clique work units (see k5_chunk)
    int k5_light;              // 5-cliques: out-degrees up to this take the one-word-row loop
    int k5_wave_words;         // 5-cliques: rows up to this many words take a wave per b
    int k5_dense_pct;          // 5-cliques: density (percent) from which the complement count is used
    int wheel_split_deg;       // wheels: hubs above this degree are split into rim tasks
    int four_range_deg;        // 4-cycles: tops above this degree are split into key-range tasks
    int pairs_hub_r;           // pattern 17: hub ranks of the hub-pair product (0: off, -1: by n)
    int pairs_hub_used;        // hub ranks the last pair pass used (0: no product)
    bool hub_w16;              // its W table holds 16-bit entries (every degree below 2^16)
    int wheel_dense_deg;       // wheels: hubs from this degree may take the product (0: never)
    int wheel_dense_ratio;     // wheels: multiply-adds one walk visit is worth
    std::vector<int32_t> wd_degs;   // row offsets of the latest ranks (for the chosen hubs)
    std::vector<uint8_t> wd_flags;  // their chosen flags (the source of an asynchronous copy)
    int32_t wd_base;           // rank of wd_degs[0]
    size_t wd_cap;             // bytes of the matrix buffer the chosen hubs go through
    int k4_dense_dplus;        // 4-cliques: vertices from this out-degree take the product (0: never)
    size_t k4_cap;             // bytes of the B_a / C_a buffer of the chosen vertices
    std::vector<int32_t> k4_ids;    // the chosen vertices (the source of an asynchronous copy)
    int pairs_hub_q;           // pattern 17: hub apexes that make an edge dense
    int five_order;            // 5-cycles of one graph: 0 Y table when maxdeg < 2^16, 1 Wnt table
    size_t dev_mem;            // device memory in bytes
    // tuning: parameters in use, forced ones, the table
    esc_params params;
    bool forced;
    esc_params force;
    uint32_t tune_key;
    int tune_used;
    uint32_t tune_keys[TUNE_SLOTS];
    esc_params tune_vals[TUNE_SLOTS];
    // esc_count_subgraphs_noalloc: during such a call every buffer is carved
    // from this fixed device region (bump pointer, never freed) instead of
    // being allocated
    char *arena;
    size_t arena_size, arena_used;
    // time slices of the per-source kernels (wall-clock ticks, 0 = none):
    // ESC_SLICE_MS in the environment, or 30 s when ESC_TRACE is set
    uint64_t slice_ticks;
    bool trace;                // report stages and slices to stderr (ESC_TRACE at creation)
};

// Workgroups of the per-source kernels (4-cycles, pair passes, 5-cycles):
// wg_per_cu per CU (two, one when the tables of a large graph would take too
// much memory); each owns dense tables of tab_n entries in B_WG_SCRATCH.
inline int pair_wgs(const esc_ctx *c) { return c->wg_per_cu * c->num_cu; }
// The 4-cycle and pattern 13/17 kernels gain more from a large LDS slab than
// from a third workgroup per CU: at most two per CU.
inline int slab_wgs_per_cu(const esc_ctx *c) { return c->wg_per_cu < 2 ? c->wg_per_cu : 2; }

// LDS words per slab for a per-source kernel with `nslabs` slabs, at most
// `cap`, so that wgs_per_cu workgroups fit in one CU's LDS next to the
// kernel's static arrays.
inline int32_t slab_words(const esc_ctx *c, int wgs_per_cu, int nslabs, int32_t cap, int static_bytes) {
    int64_t w = ((int64_t)c->max_lds / wgs_per_cu - static_bytes) / (4 * nslabs);
    if (w > cap) w = cap;
    if (w > c->tab_n) w = c->tab_n;
    if (w < 0) w = 0;
    return (int32_t)w;
}

// blocks for a grid-stride kernel over `items`: enough to cover them, at most
// per_cu per compute unit
inline int grid_cap(const esc_ctx *c, int64_t items, int threads, int per_cu = 16) {
    int64_t b = (items + threads - 1) / threads;
    const int64_t cap = (int64_t)c->num_cu * per_cu;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

inline GMap gmap_of(const esc_ctx *c) {
    GMap g;
    g.vg = c->G ? (const int32_t *)c->buf[B_VGRAPH] : nullptr;
    g.voff = c->G ? (const int64_t *)c->buf[B_GOFF] : nullptr;
    g.n = c->n;
    return g;
}

// Grow-only device buffer; returns nullptr on failure (status set by caller).
void *ctx_buf(esc_ctx *c, Buf b, size_t bytes);
// Bytes held by a buffer; release one (it is allocated again on next use).
size_t ctx_held(const esc_ctx *c, Buf b);
void ctx_release(esc_ctx *c, Buf b);
// Device bytes still free for the call's buffers: the device's free memory,
// or what is left of the fixed region of a no-allocation call.
esc_status ctx_free_bytes(esc_ctx *c, size_t *out);
// Release the buffers listed when the device has less than 64 GiB free
// (a graph whose triangle lists fill the device): a stage's large scratch
// then goes back before the next stage sizes its own.
esc_status ctx_release_if_short(esc_ctx *c, std::initializer_list<Buf> bufs);
esc_status ctx_check(hipError_t e);

// B_WORK layout: [0] W++, [1] W+-, [2 + s] visits of stage s (see esc_last_profile),
// [12] W, [13] 3T, [14] D summed over the graphs of a batched call,
// [16] sum over arcs a->b of (d+(a)-1) d+(b) (the directed 3-paths and T),
// [17] directed bipyramids, [18] W (both from the degree order)
#define WORK_VISITS 2
#define WORK_DP 16
#define WORK_DBP 17
#define WORK_W 18
#define WORK_WORDS 32

#define ESC_TRY(x) do { esc_status _s = (x); if (_s != ESC_OK) return _s; } while (0)
#define HIP_TRY(x) do { hipError_t _e = (x); if (_e != hipSuccess) return ESC_EDEVICE; } while (0)

// ESC_TRACE=1 in the environment when a context is created: its calls report
// every stage and slice to stderr
bool trace_env();

// A per-source kernel taking tasks from the shared counter `counter` (see
// slice_grab): launch(ticks) enqueues one launch.  Without slices, one
// launch with no limit.  With them, launches follow each other until a
// workgroup has seen the counter run out (*done, zeroed here), each one
// reporting its progress under ESC_TRACE, so that no launch runs much
// longer than a slice.
template <class Launch>
esc_status run_sliced(esc_ctx *c, const char *name, int *done, const int *counter, Launch launch) {
    if (c->slice_ticks == 0) return launch((uint64_t)0);
    hipStream_t st = c->stream;
    HIP_TRY(hipMemsetAsync(done, 0, sizeof(int), st));
    for (int part = 1;; part++) {
        ESC_TRY(launch(c->slice_ticks));
        int h[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(&h[0], done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&h[1], counter, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h[0]) return ESC_OK;
        if (c->trace) {
            fprintf(stderr, "esc: %s slice %d ended, %d grabs taken\n", name, part, h[1]);
            fflush(stderr);
        }
    }
}

// the walk of stage s has been enqueued: its products follow
inline esc_status mark_walk_end(esc_ctx *c, int s) {
    if (hipEventRecord(c->ev_walk[s], c->stream) != hipSuccess) return ESC_EDEVICE;
    c->walk_rec[s] = true;
    return ESC_OK;
}

// pipeline stages (each returns ESC_OK or an error)
esc_status stage_orient(esc_ctx *c, const int32_t *d_rp, const int32_t *d_col);
esc_status stage_triangles(esc_ctx *c);
esc_status stage_four(esc_ctx *c, bool per_edge_c4);
esc_status stage_pairs(esc_ctx *c);
esc_status stage_wheels(esc_ctx *c);
esc_status stage_cycles(esc_ctx *c);
esc_status stage_k4_triangles(esc_ctx *c);
esc_status stage_k5(esc_ctx *c);
esc_status stage_reduce(esc_ctx *c);
esc_status stage_combine(esc_ctx *c, esc_u128 *host_out, const int32_t *d_inv4, const int32_t *d_inv5);
esc_status stage_combine_batched(esc_ctx *c);
esc_status batched_copy_u64(esc_ctx *c, uint64_t *host_out, uint8_t *host_overflow, int *any_overflow);
esc_status batched_copy_u128(esc_ctx *c, esc_u128 *host_out);

// End of a call (api.hip): stage times, work counters, scratch marked clean.
// w, t3, d are the single-graph totals; a batch reads them from B_WORK.
esc_status call_finish(esc_ctx *c, uint64_t w, uint64_t t3, uint64_t d);

// A batch through the pipeline up to the device-side combine (api.hip); the
// rows are then copied out with batched_copy_u64 / batched_copy_u128.
esc_status run_batched_device(esc_ctx *c, int32_t G, const int64_t *vtx_off, const int64_t *arc_off,
                              const int32_t *row_ptr, const int32_t *col, int k, uint32_t flags, void *stream);
esc_status combine_tables(int32_t *host_inv4, int32_t *host_inv5);
esc_status stage_fragments_out(esc_ctx *c, uint64_t *tri_v, uint64_t *c4_v, uint64_t *k4_v,
                               uint64_t *tri_e, uint64_t *c4_e, uint64_t *k4_e);

// simple sorted symmetric CSR from any input CSR (canon.hip)
esc_status canonicalize(esc_ctx *c, int32_t n, const int32_t *d_rp, const int32_t *d_col, const int32_t **rp_out,
                        const int32_t **col_out, int64_t *m2_out);

// generic device primitives (orient.hip)
esc_status dev_exclusive_scan_i64(esc_ctx *c, const int64_t *in, int64_t *out, int64_t n);
// Tasks of a per-vertex pass numbered by the offsets toff (n + 1 entries,
// vertex v owns tasks [toff[v], toff[v+1])): *ntasks = toff[n] (read back to
// the host) and *owner[u] = the vertex of task u, on the device.
esc_status dev_task_owner(esc_ctx *c, int32_t n, const int64_t *toff, int64_t *ntasks, int32_t **owner);
esc_status dev_segsort_u32(esc_ctx *c, uint32_t *keys, const int64_t *seg_off, int64_t nseg,
                           int32_t maxlen);
