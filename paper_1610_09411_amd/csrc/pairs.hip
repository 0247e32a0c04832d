// Pair-level sums (Thm 5cutwed with the algorithm of Thm 5formula) and
// 5-cycles (Thm 5cycle).
//
//  * pattern 13 and 17: for every source i and every j after i,
//      W(i,j) = common neighbours (2-step search from i),
//      D(i,j) = edges inside the common neighbourhood, generated from a
//               triangle (i,k,l) followed by a triangle (k,l,j);
//    sum C(W,3) and sum (W-2) D over the pairs.
//  * pattern 18 (wheel, hub h): the 4-cycles inside G[N(h)], counted at their
//    latest rim vertex i like Thm 4cycle: for j before i in N(h),
//    c = #{l in N(h) & N(i) & N(j), l before i}, and sum C(c,2).  Keys j are
//    positions inside the row of h, so the table is dense and small.
//  * 5-cycles: sum over ordered pairs of P(i,j) Wnt(i,j) where P counts
//    directed 3-paths i <- a -> b -> j and Wnt the common neighbours not after
//    both i and j.  Per source i this is summed as
//      sum_b X(i,b) * sum_{j in N+(b)} Wnt(i,j),   X(i,b) = |N-(i) & N-(b)|,
//    which visits each distinct (i,b) once instead of every 3-path.
//
// Every per-source table is a dense per-workgroup array over the ranks of
// the source's graph, reset through a list of touched keys.
#include <vector>
#include "device.h"
#include "ctx.h"
#include "tiles.h"

// ------------------------------------------------------- patterns 13 and 17
//
// Every unordered pair {i, j} is taken from its earlier vertex i (the source)
// and keyed by the later one, j > i: the later endpoint of a wedge is a hub
// far more often than the earlier one, so most keys fall in the latest ranks.
// Keys in the latest `slab` ranks of the graph are counted in an LDS array,
// the rest in the workgroup's dense table (relative to the graph's start).
// The tips of diamonds are mostly hubs as well, so the diamond gathers stay
// in LDS too.

template <bool IDS>
__global__ void __launch_bounds__(512) k_pairs_wd(int32_t n, const int32_t *off, const int32_t *adj,
                                                  const int32_t *rev, const int64_t *aoff, const uint32_t *aa,
                                                  const int32_t *av, uint32_t *tab_all, int32_t *touch_all,
                                                  int32_t tab_n, int chunk, GMap gm, int *task, int32_t slab,
                                                  int32_t pw_words, unsigned long long *acc,
                                                  unsigned long long *visits, uint64_t slice_ticks, int *done,
                                                  int32_t hub0, int32_t hub_r, const int32_t *did,
                                                  void *wtop, int w16) {
    extern __shared__ uint32_t sl[];
    uint64_t nvis = 0;
    const uint64_t slice_end = slice_end_of(slice_ticks);
    __shared__ int pref[513], tmp[16];
    __shared__ int64_t beg[513];
    __shared__ int s_i, s_nt;
    __shared__ u128 red[2 * 8];
    __shared__ int64_t wsa[8][64];
    __shared__ int32_t wse[8][64], wsi[8][64];
    const int ids[2] = {AC_N13, AC_N17};
    uint32_t *Wt = tab_all + (size_t)blockIdx.x * tab_n;
    int32_t *touch = touch_all + (size_t)blockIdx.x * tab_n;
    u128 sv[2] = {0, 0};   // pattern 13, pattern 17
    int gcur = -1;
    if (pw_words > 0) {
        // a batch of small graphs: one source per wave, W(i,.) in the wave's
        // own LDS table over the keys after i in its graph (pw_words words),
        // cleared per source, so no touched list and no workgroup barrier
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
        uint32_t *wt = sl + (size_t)wid * pw_words;
        int (*wrun)[64] = (int (*)[64])pref;   // per wave: inclusive entry counts of 64 arcs
        int wgc = -1;   // graph of the wave's sums
        for (;;) {
            if (threadIdx.x == 0) s_i = slice_grab(task, slice_end);
            __syncthreads();
            const int gi = s_i;
            const int64_t t0 = (int64_t)gi * chunk * nwv;
            __syncthreads();   // s_i is read by every thread before it is taken again
            if (t0 >= n) {
                if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
                break;
            }
            const int64_t t1 = t0 + (int64_t)chunk * nwv < n ? t0 + (int64_t)chunk * nwv : n;
            for (int64_t t = t0 + wid; t < t1; t += nwv) {
                const int32_t i = n - 1 - (int32_t)t;
                const int32_t oi = off[i], ei = off[i + 1];
                if (ei - oi < 3) continue;   // d(i) <= 2 adds nothing (as below)
                const int g = gm.graph(i);
                if (g != wgc) {
                    if (wgc >= 0) wave_flush_runs<2>(sv, wgc, acc, ACC_STRIDE, ids);
                    wgc = g;
                }
                const int32_t ge = gm.end(g);
                const int shift = count_shift(ei - oi);
                const int cb = 32 >> shift;
                const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
                const int32_t nwd = ((ge - i - 1) + (1 << shift) - 1) >> shift;   // words of keys (i, ge)
                for (int q = lane; q < nwd; q += 64) wt[q] = 0;
                wave_sync();
                // W(i,j), j after i: k in N(i), j in the suffix of N(k) after i
                for (int32_t pb = oi; pb < ei; pb += 64) {
                    const int32_t p = pb + lane;
                    int64_t a0 = 0, a1 = 0;
                    if (p < ei) { a0 = rev[p] + 1; a1 = off[adj[p] + 1]; }
                    nvis += (uint64_t)(a1 - a0);
                    wave_walk(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return adj[q]; },
                              [&](int32_t j) {
                                  const int32_t idx = j - i - 1;
                                  atomicAdd(&wt[idx >> shift], 1u << ((idx & ((1 << shift) - 1)) * cb));
                              });
                }
                wave_sync();
                // diamonds with tips i and j: the entries l after k of the
                // lists of the arcs (i,k), 64 arcs at a time numbered in one
                // run (a lane per entry), then the suffix of the list of (k,l)
                // after i.  Non-empty suffixes are gathered by ballot into the
                // wave's staging array (start << 24 | length: lists of a batch
                // of small graphs hold fewer than 2^40 entries, a suffix
                // fewer than 2^24) and walked by the wave 64 at a time.
                uint64_t acc17 = 0;
                uint64_t *stg = (uint64_t *)beg + wid * 64;   // beg is unused by this path
                const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                int staged = 0;   // wave-uniform
                auto walk_staged = [&]() {
                    wave_sync();   // staged suffixes visible to the wave
                    int64_t a0 = 0, a1 = 0;
                    if (lane < staged) {
                        const uint64_t v = stg[lane];
                        a0 = (int64_t)(v >> 24);
                        a1 = a0 + (int64_t)(v & 0xFFFFFFu);
                    }
                    wave_walk(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return apex_at<IDS>(av, adj, aa, q); },
                              [&](int32_t j) {
                                  const int32_t idx = j - i - 1;
                                  acc17 += (uint64_t)((wt[idx >> shift] >> ((idx & ((1 << shift) - 1)) * cb)) & cmask) - 2;
                              });
                    staged = 0;   // the walk ends with a wave_sync: the array is free
                };
                for (int32_t pb = oi; pb < ei; pb += 64) {
                    const int32_t pl = pb + lane;
                    const int cnt = pl < ei ? (int)(aoff[pl + 1] - aoff[pl]) : 0;
                    int incl = cnt;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int y = __shfl_up(incl, o);
                        if (lane >= o) incl += y;
                    }
                    const int total = __shfl(incl, 63);
                    wrun[wid][lane] = incl;
                    wave_sync();
                    int y = 0;
                    for (int tb = 0; tb < total; tb += 64) {
                        const int f = tb + lane;
                        int64_t a0 = 0, a1 = 0;
                        if (f < total) {
                            while (wrun[wid][y] <= f) y++;
                            const int32_t pk = pb + y;
                            const int64_t e0 = aoff[pk];
                            const int64_t x = e0 + (f - (wrun[wid][y] - (int)(aoff[pk + 1] - e0)));
                            if (aa[x] > (uint32_t)pk) {   // l > k, compared as arcs of row i (as below)
                                const uint32_t ki = (uint32_t)rev[pk];   // arc (k,i) in row k
                                const int32_t qkl = (int32_t)aa[aoff[ki] + (x - e0)];   // arc (k,l) in row k
                                int64_t lo2 = aoff[qkl], hi2 = aoff[qkl + 1];
                                a1 = hi2;
                                while (lo2 < hi2) { int64_t mid = (lo2 + hi2) >> 1; if (aa[mid] <= ki) lo2 = mid + 1; else hi2 = mid; }
                                a0 = lo2;
                            }
                        }
                        nvis += (uint64_t)(a1 - a0);
                        const uint64_t m = __ballot(a1 > a0);
                        if (m == 0) continue;
                        if (staged + __popcll(m) > 64) walk_staged();
                        if (a1 > a0) stg[staged + __popcll(m & lt)] = ((uint64_t)a0 << 24) | (uint64_t)(a1 - a0);
                        staged += __popcll(m);
                    }
                    wave_sync();   // wrun is rewritten by the next 64 arcs
                }
                if (staged > 0) walk_staged();
                sv[1] += acc17;
                // sum of C(W,3) over the keys
                for (int q = lane; q < nwd; q += 64) {
                    const uint32_t x = wt[q];
                    if (x != 0) sv[0] += c3_fields(x, cb, cmask);
                }
                wave_sync();   // the table is cleared by the wave's next source
            }
        }
        if (wgc >= 0) wave_flush_runs<2>(sv, wgc, acc, ACC_STRIDE, ids);
        flush_count(nvis, visits);
        return;
    }
    if (threadIdx.x == 0) s_nt = 0;
    for (;;) {
        if (threadIdx.x == 0) s_i = slice_grab(task, slice_end);
        __syncthreads();
        const int gi = s_i;
        const int64_t t0 = task_begin(gi, chunk), tn = task_begin((int64_t)gi + 1, chunk);
        // s_i is read by every thread before it is taken again: a chunk whose
        // sources are all skipped has no other barrier before the next take
        __syncthreads();
        if (t0 >= n) {
            if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
            break;
        }
        const int32_t t1 = (int32_t)(tn < n ? tn : n);
        for (int32_t t = (int32_t)t0; t < t1; t++) {
        const int32_t i = n - 1 - t;
        const int g = gm.graph(i);
        block_switch_graph<2>(sv, gcur, g, red, acc, ACC_STRIDE, ids);
        const int32_t gb = gm.begin(g), ge = gm.end(g);
        const int32_t oi = off[i], ei = off[i + 1];
        // W(i,j) <= d(i): with d(i) <= 2 every C(W,3) is 0, and a diamond's
        // tips share both its middles, so its W - 2 is 0 too
        if (ei - oi < 3) continue;
        // W(i,j) <= d(i): counts of a low-degree source are packed 16, 8, 4
        // or 2 to a word (count_shift), so the LDS slab covers that many
        // times more latest ranks and the workgroup table touches that many
        // times fewer cache lines
        const int shift = count_shift(ei - oi);   // log2(counts per word)
        const int cb = 32 >> shift;                                        // bits per count
        const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
        const int32_t sranks = slab << shift;
        const int32_t hi0 = ge - sranks > gb ? ge - sranks : gb;           // first key held in LDS
        const int32_t ls = i + 1 > hi0 ? i + 1 : hi0;                       // LDS keys [ls, ge)
        const int32_t w_lo = (ls - hi0) >> shift, w_hi = ge > ls ? ((ge - 1 - hi0) >> shift) + 1 : w_lo;
        for (int q = w_lo + threadIdx.x; q < w_hi; q += blockDim.x) sl[q] = 0;
        __syncthreads();
#define SLAB_INC(j) atomicAdd(&sl[((j) - hi0) >> shift], 1u << ((((j) - hi0) & ((1 << shift) - 1)) * cb))
#define SLAB_GET(j) ((sl[((j) - hi0) >> shift] >> ((((j) - hi0) & ((1 << shift) - 1)) * cb)) & cmask)
#define TAB_SH(j) ((uint32_t)((((j) - gb) & ((1 << shift) - 1)) * cb))
#define TAB_INC(j) ((atomicAdd(&Wt[((j) - gb) >> shift], 1u << TAB_SH(j)) >> TAB_SH(j)) & cmask)
#define TAB_GET(j) ((Wt[((j) - gb) >> shift] >> TAB_SH(j)) & cmask)
        // W(i,j) for j after i: k in N(i), j in the suffix of N(k) after i
        for (int32_t base = oi; base < ei; base += blockDim.x) {
            int32_t p = base + threadIdx.x;
            int start = 0, len = 0;
            if (p < ei) { int32_t k = adj[p]; start = rev[p] + 1; len = off[k + 1] - start; }
            nvis += (uint64_t)len;
            lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                            [&](int, int64_t, int32_t j) {
                                if (j >= hi0) SLAB_INC(j);
                                else if (TAB_INC(j) == 0) touch[atomicAdd(&s_nt, 1)] = j;
                            });
        }
        __syncthreads();
        // a hub source keeps its row W(i, j) over the later hubs for the
        // hub-pair product (the slab holds every key from hub0 on)
        if (i >= hub0) {
            const size_t r0 = (size_t)(i - hub0) * hub_r;
            for (int32_t j = i + 1 + threadIdx.x; j < ge; j += blockDim.x) {
                const uint32_t w = j >= hi0 ? SLAB_GET(j) : TAB_GET(j);
                if (w16) ((uint16_t *)wtop)[r0 + (j - hub0)] = (uint16_t)w;   // W <= d(i) < 2^16
                else ((uint32_t *)wtop)[r0 + (j - hub0)] = w;
            }
        }
        // diamonds with tips i and j (j after i): triangles (i,k,l), k<l, then
        // apexes j of edge (k,l) after i.  The entries l of the triangle
        // lists of the arcs (i,k), up to blockDim arcs at a time, are
        // numbered in one run and dealt to the waves in turn (so a source
        // with few arcs or short lists still keeps every wave busy); each
        // lane finds one segment, the suffix of the list of (k,l) after i,
        // and the wave walks its 64 segments together.
        {
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
            for (int32_t base = oi; base < ei; base += blockDim.x) {
                const int32_t pt = base + threadIdx.x;
                const int cnt = pt < ei ? (int)(aoff[pt + 1] - aoff[pt]) : 0;
                int total;
                const int ex = block_exclusive_scan(cnt, tmp, &total);
                pref[threadIdx.x] = ex;
                if (threadIdx.x == 0) pref[blockDim.x] = total;
                __syncthreads();
                int lo = 0;   // the arc whose entries hold f: f only grows, so
                              // its search goes on from the previous arc
                for (int fb = 0; fb < total; fb += nw * 64) {
                    const int f = fb + lane * nw + wid;
                    int64_t a0 = 0, a1 = 0;
                    if (f < total) {
                        if (pref[lo + 1] <= f) {
                            int a = lo + 1, step = 1, lim = (int)blockDim.x - 1;   // pref[a] <= f
                            while (a + step <= lim && pref[a + step] <= f) { a += step; step <<= 1; }
                            int hi = a + step <= lim ? a + step - 1 : lim;
                            while (a < hi) {
                                const int mid = (a + hi + 1) >> 1;
                                if (pref[mid] <= f) a = mid; else hi = mid - 1;
                            }
                            lo = a;
                        }
                        const int32_t pk = base + lo;
                        const int64_t e0 = aoff[pk];
                        const int64_t x = e0 + (f - pref[lo]);
                        // the list of (i,k) holds the arcs (i,l) of row i and
                        // rows are sorted, so l > k is aa[x] > pk; the list of
                        // (k,l) holds arcs (k,j) of row k, so j > i is an entry
                        // after the arc (k,i) = rev[pk]: no apex is read
                        bool skip = aa[x] <= (uint32_t)pk;
                        uint32_t ki = 0;
                        int32_t qkl = 0;
                        if (!skip) {
                            ki = (uint32_t)rev[pk];
                            qkl = (int32_t)aa[aoff[ki] + (x - e0)];   // arc (k,l) in row k
                        }
                        // a hub source leaves the edges with many hub apexes
                        // to the hub-pair product (every j after it is a hub);
                        // such an edge has a number at its arc in the row of
                        // its earlier end
                        if (!skip && i >= hub0) skip = did[qkl] >= 0;
                        if (!skip) {
                            int64_t lo2 = aoff[qkl], hi2 = aoff[qkl + 1];
                            a1 = hi2;
                            while (lo2 < hi2) { int64_t mid = (lo2 + hi2) >> 1; if (aa[mid] <= ki) lo2 = mid + 1; else hi2 = mid; }
                            a0 = lo2;
                        }
                    }
                    nvis += (uint64_t)(a1 - a0);
                    uint64_t acc17 = 0;
                    // twelve steps in flight: each element of compact lists is
                    // two dependent loads
                    wave_walk<IDS ? 8 : 12>(a0, a1, wsa[wid], wse[wid], wsi[wid],
                              [&](int64_t q) { return apex_at<IDS>(av, adj, aa, q); },
                              [&](int32_t j) { acc17 += (uint64_t)(j >= hi0 ? SLAB_GET(j) : TAB_GET(j)) - 2; });
                    sv[1] += acc17;
                }
                __syncthreads();   // pref is rewritten by the next batch of arcs
            }
        }
        const int nt = s_nt;
        for (int q = threadIdx.x; q < nt; q += blockDim.x) {
            const int32_t j = touch[q];
            // other counts of the word may be reset concurrently
            const uint32_t old = atomicAnd(&Wt[(j - gb) >> shift], ~(cmask << TAB_SH(j)));
            sv[0] += c3((old >> TAB_SH(j)) & cmask);
        }
        if (ei - oi >= 3)   // W(i,j) <= d(i): below 3 no pair has C(W,3) > 0
            for (int q = w_lo + threadIdx.x; q < w_hi; q += blockDim.x) {
                const uint32_t x = sl[q];
                if (x != 0) sv[0] += c3_fields(x, cb, cmask);
            }
#undef SLAB_INC
#undef SLAB_GET
#undef TAB_SH
#undef TAB_INC
#undef TAB_GET
        __syncthreads();
        if (threadIdx.x == 0) s_nt = 0;   // next read of s_nt is behind a barrier
        }
    }
    if (gcur >= 0) block_flush_u128<2>(sv, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    flush_count(nvis, visits);
}

// ------------------------------------------------------------ pattern 18

// Hub h, each neighbour i of h taken as the latest rim vertex: l runs over
// the triangle list of arc (h,i) below i, j over the triangle list of arc
// (h,l) below i; key = position of j in the row of h, and C(count,2) summed
// over keys counts the rim 4-cycles with latest vertex i (summed as the
// count before each increment).  Counts live in LDS: a count is below d(h),
// so two share a word when d(h) < 2^16 (16 bits each; one 32-bit atomic
// adds 1 << 16 for odd keys), else one count per word.
//
// Hubs with d(h) > wq (the largest hub of the per-wave mode) come first as
// tasks of (a block of rim vertices, a range of keys): blocks of WHEEL_RIMS
// rim vertices above split_deg neighbours (else all of them), key ranges of
// `wk` keys (wk / 2 for 32-bit counts), so every table fits the LDS of a
// workgroup whatever d(h).  A task reads from each list of (h,l) only the run
// of keys in its range below i (the lists are sorted by position in the row
// of h: two binary searches find it).  Tasks are numbered per hub in toff,
// latest hubs first: every workgroup of the chip works on the same few hubs
// at a time, so their triangle lists, re-read for every rim vertex, stay in
// each XCD's L2.  The smaller hubs follow, one per workgroup, each wave
// taking its own rim vertices with its own table and no workgroup barrier
// per rim vertex.
#define WHEEL_WAVES 8          // most waves per workgroup of the wheel pass (a launch may use fewer)
#define WHEEL_RIMS 16          // rim vertices per task of a large hub
#define WHEEL_TINY 32          // batches: hubs up to this degree are taken whole by one wave
#define WHEEL_TINY_WORDS (WHEEL_TINY * WHEEL_TINY / 2)   // its table: 16-bit counts of (rim, key)

// rim vertices per task of hub with d neighbours: all of them up to split_deg
__device__ inline int32_t wheel_rims(int32_t d, int32_t split_deg) { return d > split_deg ? WHEEL_RIMS : d; }
// keys per range of a hub with d neighbours (16-bit counts below 2^16)
__device__ inline int32_t wheel_keys(int32_t d, int32_t wk) { return d < 65536 ? wk : wk / 2; }

// hubs from rank wd_lo on with wflag set are counted by the product (below)
__device__ inline bool wheel_dense(int32_t h, int32_t wd_lo, const uint8_t *wflag) {
    return h >= wd_lo && wflag[h - wd_lo];
}

__global__ void k_wheel_tasks(int32_t n, const int32_t *off, int32_t wq, int32_t split_deg, int32_t wk,
                              int32_t wd_lo, const uint8_t *wflag, int64_t *len) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t d = off[v + 1] - off[v];
        const int64_t nr = (d + wheel_rims(d, split_deg) - 1) / wheel_rims(d, split_deg);
        const int64_t nk = (d + wheel_keys(d, wk) - 1) / wheel_keys(d, wk);
        len[v] = d > wq && !wheel_dense(v, wd_lo, wflag) ? nr * nk : 0;
    }
}

template <bool IDS>
__global__ void __launch_bounds__(64 * WHEEL_WAVES) k_wheels(int32_t n, const int32_t *off, const int32_t *adj,
                                                const int64_t *aoff, const uint32_t *aa, const int32_t *av,
                                                int32_t wq, int32_t wk, int32_t tab_words, const int64_t *toff,
                                                const int32_t *town,
                                                int64_t nbig, int *task_big, int chunk, int32_t split_deg,
                                                GMap gm, int *task, int tiny, unsigned long long *acc,
                                                unsigned long long *visits, uint64_t slice_ticks, int *done,
                                                int32_t wd_lo, const uint8_t *wflag) {
    uint64_t nvis = 0;
    const uint64_t slice_end = slice_end_of(slice_ticks);
    extern __shared__ uint32_t dyn[];
    __shared__ int s_h, s_r, s_ntw[WHEEL_WAVES];
    __shared__ u128 red[WHEEL_WAVES];   // one sum per wave (block_flush_u128)
    __shared__ int64_t wsa[WHEEL_WAVES][64];
    __shared__ int32_t wse[WHEEL_WAVES][64], wsi[WHEEL_WAVES][64];
    __shared__ int32_t wkb[WHEEL_WAVES][64];   // tiny hubs: key base (rim index * d(h)) of each segment
    const int ids[1] = {AC_N18};
    u128 s18[1] = {0};
    int gcur = -1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t *lcnt = dyn;   // the key range of a large-hub task
    // zero at the start; every rim vertex leaves the table zero again
    for (int q = threadIdx.x; q < tab_words; q += blockDim.x) lcnt[q] = 0;
    __syncthreads();

    // large hubs: tasks of WHEEL_RIMS rim vertices
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t u = nbig - 1 - slice_grab(task_big, slice_end);
            int32_t v = -1;
            if (u >= 0) {
                v = town[u];
                s_r = (int)(u - toff[v]);
            }
            s_h = v;
        }
        __syncthreads();
        const int32_t h = s_h;
        const int rtask = s_r;
        __syncthreads();   // s_h, s_r are read by every thread before they are taken again
        if (h < 0) break;
        block_switch_graph<1>(s18, gcur, gm.graph(h), red, acc, ACC_STRIDE, ids);
        const int32_t oh = off[h], dh = off[h + 1] - oh;
        const int32_t rims = wheel_rims(dh, split_deg), kr = wheel_keys(dh, wk);
        const int32_t nk = (dh + kr - 1) / kr;
        const int32_t r0 = (rtask / nk) * rims;
        const int32_t r1 = r0 + rims < dh ? r0 + rims : dh;
        const int32_t k0 = (rtask % nk) * kr;   // keys [k0, k0 + kr) of this task
        const bool wide = dh >= 65536;          // 32-bit counts
        for (int32_t pi = oh + r0; pi < oh + r1; pi++) {
            const int32_t ip = pi - oh;         // position of i: its keys lie below it
            if (ip <= k0) continue;
            const int32_t k1 = ip < k0 + kr ? ip : k0 + kr;
            const int64_t l0 = aoff[pi], l1 = aoff[pi + 1];
            if (l1 - l0 < 2) continue;   // a rim 4-cycle needs two triangles on (h,i)
            // entries l of list(h,i) below i (positions below ip)
            int64_t lo = l0, hi = l1;
            while (lo < hi) { int64_t mid = (lo + hi) >> 1; if ((int32_t)aa[mid] - oh < ip) lo = mid + 1; else hi = mid; }
            const int nl = (int)(lo - l0);
            if (nl == 0) continue;
            // each wave takes entries l; its lanes stride over the run of
            // the list of (h,l) with keys in [k0, k1)
            for (int xb = 0; xb < nl; xb += nw * 64) {
                // each lane finds one segment; entries are dealt to the
                // waves in turn, so a short list of l still keeps every
                // wave busy
                const int x = xb + lane * nw + wid;
                int64_t b0 = 0, b1 = 0;
                if (x < nl) {
                    const int32_t qhl = (int32_t)aa[l0 + x];       // arc (h,l) in row h
                    int64_t e0 = aoff[qhl], e1 = aoff[qhl + 1];
                    if (k0 > 0) {
                        int64_t hi2 = e1;
                        while (e0 < hi2) { int64_t mid = (e0 + hi2) >> 1; if ((int32_t)aa[mid] - oh < k0) e0 = mid + 1; else hi2 = mid; }
                    }
                    b0 = e0;
                    int64_t lo2 = e0;
                    while (lo2 < e1) { int64_t mid = (lo2 + e1) >> 1; if ((int32_t)aa[mid] - oh < k1) lo2 = mid + 1; else e1 = mid; }
                    b1 = lo2;
                }
                nvis += (uint64_t)(b1 - b0);
                // sum over keys of C(count,2) = sum over increments of the
                // count before it
                uint64_t olds = 0;
                if (!wide)
                    wave_walk_act(b0, b1, wsa[wid], wse[wid], wsi[wid],
                                  [&](int64_t q) { return (int32_t)aa[q] - oh - k0; },
                                  [&](int32_t key) { return atomicAdd(&lcnt[key >> 1], 1u << ((key & 1) << 4)); },
                                  [&](int32_t key, uint32_t old) { olds += (old >> ((key & 1) << 4)) & 0xFFFFu; });
                else
                    wave_walk_act(b0, b1, wsa[wid], wse[wid], wsi[wid],
                                  [&](int64_t q) { return (int32_t)aa[q] - oh - k0; },
                                  [&](int32_t key) { return atomicAdd(&lcnt[key], 1u); },
                                  [&](int32_t, uint32_t old) { olds += old; });
                s18[0] += olds;
            }
            __syncthreads();
            // the table back to zero: every key touched lies in [k0, k1)
            const int32_t words = wide ? k1 - k0 : (k1 - k0 + 1) / 2;
            for (int q = threadIdx.x; q < words; q += blockDim.x) lcnt[q] = 0;
            __syncthreads();
        }
    }

    // smaller hubs: one per workgroup, one table per wave
    const int32_t rw = (wq + 1) / 2;   // words of a wave's table, and of its touched list
    uint32_t *wc = dyn + (size_t)wid * 2 * rw;
    uint16_t *wt = (uint16_t *)(wc + rw);
    // tiny hubs: the wave's one-wave table when it is large enough (the wave
    // uses either, never both at once), else a table after those tables
    uint32_t *tt = 2 * rw >= WHEEL_TINY_WORDS ? wc : dyn + (size_t)nw * 2 * rw + (size_t)wid * WHEEL_TINY_WORDS;
    u128 ts[1] = {0};   // tiny hubs: the wave's sums, for graph tg
    int tg = -1;
    for (;;) {
        if (threadIdx.x == 0) s_h = slice_grab(task, slice_end);
        __syncthreads();
        const int gi = s_h;
        const int64_t t0 = task_begin(gi, chunk), tn = task_begin((int64_t)gi + 1, chunk);
        if (t0 >= n) {
            if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
            break;
        }
        const int32_t t1 = (int32_t)(tn < n ? tn : n);
        __syncthreads();   // s_h is read by every thread before it is taken again
        for (int32_t t = (int32_t)t0; t < t1; t++) {
            const int32_t h = n - 1 - t;
            const int32_t oh = off[h], dh = off[h + 1] - oh;
            // large hubs are done; a wheel hub has 4 neighbours
            if (dh > wq || dh < 3 || wheel_dense(h, wd_lo, wflag)) continue;
            if (dh <= tiny) {
                // one wave takes the whole hub: counts keyed by (rim index a,
                // key), d(h)^2 16-bit counts in the wave's own table, so the
                // rim vertices need no reset between them and all their
                // (i, l) segments are walked as runs of 64
                if ((t - (int32_t)t0) % nw != wid) continue;
                const int g = gm.graph(h);
                if (g != tg) {
                    if (tg >= 0) wave_flush_runs<1>(ts, tg, acc, ACC_STRIDE, ids);
                    tg = g;
                }
                for (int q = lane; q < (dh * dh + 1) / 2; q += 64) tt[q] = 0;
                // lane a < d(h): rim vertex i = adj[oh + a] and its entries l below i
                // (lists hold arcs of row h, so "below i" is "before its arc")
                const uint32_t ia = (uint32_t)(oh + lane);   // arc (h,i) in row h
                long long la = 0;
                int na = 0;
                if (lane < dh) {
                    const int64_t l0 = aoff[oh + lane], l1 = aoff[oh + lane + 1];
                    la = l0;
                    if (l1 - l0 >= 2) {   // a rim 4-cycle needs two triangles on (h,i)
                        int64_t lo = l0, hi = l1;
                        while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (aa[mid] < ia) lo = mid + 1; else hi = mid; }
                        na = (int)(lo - l0);
                    }
                }
                int incl = na;
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                const int np = __shfl(incl, 63);   // (rim vertex, entry) pairs of the hub
                wave_sync();   // the table is cleared
                uint64_t olds = 0;   // the counts before each increment
                for (int xb = 0; xb < np; xb += 64) {
                    const int x = xb + lane;
                    // rim index a of pair x: the first lane with incl > x (every
                    // lane takes part in the shuffles)
                    int a = 0;
                    for (int sb = 32; sb > 0; sb >>= 1)
                        if (__shfl(incl, a + sb - 1) <= x) a += sb;
                    a = a < 63 ? a : 63;
                    const uint32_t iA = (uint32_t)(oh + a);   // arc (h,i) of rim index a
                    const long long lA = __shfl(la, a);
                    const int eA = __shfl(incl, a) - __shfl(na, a);   // pairs before rim index a
                    int64_t b0 = 0, b1 = 0;
                    if (x < np) {
                        const int32_t qhl = (int32_t)aa[lA + (x - eA)];   // arc (h,l) in row h
                        b0 = aoff[qhl];
                        int64_t lo2 = b0, hi2 = aoff[qhl + 1];
                        while (lo2 < hi2) { int64_t mid = (lo2 + hi2) >> 1; if (aa[mid] < iA) lo2 = mid + 1; else hi2 = mid; }
                        b1 = lo2;
                    }
                    nvis += (uint64_t)(b1 - b0);
                    wkb[wid][lane] = a * dh;   // visible to the wave after the walk's own wave_sync
                    wave_walk_seg(b0, b1, wsa[wid], wse[wid], wsi[wid],
                                  [&](int64_t q) { return (int32_t)aa[q] - oh; },
                                  [&](int y, int64_t, int32_t j) {
                                      const int32_t key = wkb[wid][y] + j;
                                      const uint32_t old = atomicAdd(&tt[key >> 1], 1u << ((key & 1) << 4));
                                      olds += (old >> ((key & 1) << 4)) & 0xFFFFu;
                                  });
                }
                ts[0] += olds;
                wave_sync();   // the table is cleared by the wave's next tiny hub
                continue;
            }
            block_switch_graph<1>(s18, gcur, gm.graph(h), red, acc, ACC_STRIDE, ids);
            for (int q = lane; q < (dh + 1) / 2; q += 64) wc[q] = 0;
            wave_sync();
            for (int32_t pi = oh + wid; pi < oh + dh; pi += nw) {
                const int64_t l0 = aoff[pi], l1 = aoff[pi + 1];   // rim vertex i = adj[pi]
                if (l1 - l0 < 2) continue;
                int64_t lo = l0, hi = l1;   // entries before the arc (h,i): apexes below i
                while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (aa[mid] < (uint32_t)pi) lo = mid + 1; else hi = mid; }
                const int nl = (int)(lo - l0);
                if (nl == 0) continue;
                if (lane == 0) s_ntw[wid] = 0;
                wave_sync();
                for (int xb = 0; xb < nl; xb += 64) {
                    const int x = xb + lane;
                    int64_t b0 = 0, b1 = 0;
                    if (x < nl) {
                        const int32_t qhl = (int32_t)aa[l0 + x];       // arc (h,l) in row h
                        b0 = aoff[qhl];
                        int64_t lo2 = b0, hi2 = aoff[qhl + 1];
                        while (lo2 < hi2) { int64_t mid = (lo2 + hi2) >> 1; if (aa[mid] < (uint32_t)pi) lo2 = mid + 1; else hi2 = mid; }
                        b1 = lo2;
                    }
                    nvis += (uint64_t)(b1 - b0);
                    uint64_t olds = 0;   // as above: the counts before each increment
                    wave_walk_act(b0, b1, wsa[wid], wse[wid], wsi[wid],
                                  [&](int64_t q) { return (int32_t)aa[q] - oh; },
                                  [&](int32_t key) { return atomicAdd(&wc[key >> 1], 1u << ((key & 1) << 4)); },
                                  [&](int32_t key, uint32_t old) {
                                      const uint32_t c = (old >> ((key & 1) << 4)) & 0xFFFFu;
                                      olds += c;
                                      if (c == 0) wt[atomicAdd(&s_ntw[wid], 1)] = (uint16_t)key;
                                  });
                    s18[0] += olds;
                }
                const int nt = s_ntw[wid];
                for (int q = lane; q < nt; q += 64) {
                    const int32_t key = wt[q];
                    atomicAnd(&wc[key >> 1], ~(0xFFFFu << ((key & 1) << 4)));
                }
                wave_sync();
            }
        }
    }
    if (tg >= 0) wave_flush_runs<1>(ts, tg, acc, ACC_STRIDE, ids);
    if (gcur >= 0) block_flush_u128<1>(s18, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    flush_count(nvis, visits);
}

// ---------------------------------------------------------------- 5-cycles

#define FIVE_WAVE_KEYS 64    // keys b from which the final sum runs as wave walks

// Keys in the latest `slab` ranks of the graph (mostly hubs: X keys are
// out-neighbours, the 3-path ends j are out-neighbours of them) use two LDS
// arrays, one for X and one for Wnt; the rest use the workgroup's tables.
// Both are reset through the touched-key lists.
// WALK: the final sum may run as wave walks; the kernel without them needs
// half the registers, so more workgroups stay resident (batches of small
// graphs, where few sources have FIVE_WAVE_KEYS keys)
template <bool WALK, bool YSUM>
__global__ void __launch_bounds__(512) k_five_cycles(int32_t n, const int32_t *off, const int32_t *adj,
                                                     const int32_t *split, uint32_t *tabX_all, uint32_t *tabW_all,
                                                     int32_t *touchX_all, int32_t *touchW_all, int32_t tab_n,
                                                     int chunk, GMap gm, int *task, int32_t slab,
                                                     int32_t pw_words, unsigned long long *acc,
                                                     unsigned long long *visits, uint64_t slice_ticks, int *done) {
    extern __shared__ uint32_t dyn[];   // [0, xslab) X, [xslab, 2 slab) Wnt or Y
    uint64_t nvis = 0;
    const uint64_t slice_end = slice_end_of(slice_ticks);
    __shared__ int pref[513], tmp[16];
    __shared__ int64_t beg[513];
    __shared__ int s_i, s_nx, s_nw;
    __shared__ u128 red[8];
    __shared__ int32_t wsi[8][64];    // wave walks: segment ends (starts alias pref, firsts alias beg)
    __shared__ uint32_t wxs[8][64];   // X(i,b) of each lane's segment
    __shared__ int32_t wkb[8][64];    // per-wave path: keys b staged for a walk of their out-rows
    const int ids[1] = {AC_CYC};
    uint32_t *Xt = tabX_all + (size_t)blockIdx.x * tab_n;
    uint32_t *Wt = tabW_all + (size_t)blockIdx.x * tab_n;
    int32_t *tx = touchX_all + (size_t)blockIdx.x * tab_n;
    int32_t *tw = touchW_all + (size_t)blockIdx.x * tab_n;
    // LDS words of the X array: half of the two arrays, or in the Y order an
    // eighth (X counts pack several per word, Y takes a word per key and
    // its reads are the many)
    const int32_t xslab = YSUM ? slab / 4 : slab;
    uint32_t *sX = dyn, *sW = dyn + xslab;
    u128 sc[1] = {0};
    int gcur = -1;
    if (pw_words > 0) {
        // a batch of small graphs: one source per wave, X(i,.) and Wnt(i,.)
        // in the wave's own LDS tables over the keys of its graph (pw_words
        // words each), cleared per source; the final sum scans the X table
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
        uint32_t *wx = dyn + (size_t)wid * 2 * pw_words, *ww = wx + pw_words;
        int64_t *wsa = beg + wid * 64;
        int32_t *wse = pref + wid * 64;
        int wgc = -1;   // graph of the wave's sums
        for (;;) {
            if (threadIdx.x == 0) s_i = slice_grab(task, slice_end);
            __syncthreads();
            const int gi = s_i;
            const int64_t t0 = (int64_t)gi * chunk * nwv;
            __syncthreads();   // s_i is read by every thread before it is taken again
            if (t0 >= n) {
                if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
                break;
            }
            const int64_t t1 = t0 + (int64_t)chunk * nwv < n ? t0 + (int64_t)chunk * nwv : n;
            for (int64_t t = t0 + wid; t < t1; t += nwv) {
                const int32_t i = n - 1 - (int32_t)t;
                const int32_t oi = off[i], si = split[i], ei = off[i + 1];
                if (si == oi) continue;   // no in-neighbour: no X key
                const int g = gm.graph(i);
                if (g != wgc) {
                    if (wgc >= 0) wave_flush_runs<1>(sc, wgc, acc, ACC_STRIDE, ids);
                    wgc = g;
                }
                const int32_t gb = gm.begin(g), ge = gm.end(g);
                const int shift = count_shift(ei - oi);
                const int cb = 32 >> shift;
                const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
                const int32_t nwd = ((ge - gb) + (1 << shift) - 1) >> shift;   // words of the graph's keys
                for (int q = lane; q < nwd; q += 64) { wx[q] = 0; ww[q] = 0; }
                wave_sync();
                auto add = [&](uint32_t *tb, int32_t x) {
                    const int32_t idx = x - gb;
                    atomicAdd(&tb[idx >> shift], 1u << ((idx & ((1 << shift) - 1)) * cb));
                };
                // X(i,b): a in N-(i), b in N+(a), b != i
                for (int32_t pb = oi; pb < si; pb += 64) {
                    const int32_t p = pb + lane;
                    int64_t a0 = 0, a1 = 0;
                    if (p < si) { const int32_t a = adj[p]; a0 = split[a]; a1 = off[a + 1]; }
                    nvis += (uint64_t)(a1 - a0);
                    wave_walk(a0, a1, wsa, wse, wsi[wid], [&](int64_t q) { return adj[q]; },
                              [&](int32_t b) { if (b != i) add(wx, b); });
                }
                // Wnt(i,j): c in N(i); all of N(c) when c is before i, else only N+(c)
                for (int32_t pb = oi; pb < ei; pb += 64) {
                    const int32_t p = pb + lane;
                    int64_t a0 = 0, a1 = 0;
                    if (p < ei) {
                        const int32_t cv = adj[p];
                        a0 = cv < i ? off[cv] : split[cv];
                        a1 = off[cv + 1];
                    }
                    nvis += (uint64_t)(a1 - a0);
                    wave_walk(a0, a1, wsa, wse, wsi[wid], [&](int64_t q) { return adj[q]; },
                              [&](int32_t j) { if (j != i) add(ww, j); });
                }
                wave_sync();
                // sum_b X(i,b) sum_{j in N+(b)} Wnt(i,j): the keys b with
                // X(i,b) > 0 are gathered (ballot over 64 keys at a time) into
                // the wave's staging array, and each full batch of them has
                // its out-rows walked by the wave as one run
                u128 part = 0;
                const int32_t nk = ge - gb;
                const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                int staged = 0;   // wave-uniform
                auto walk_staged = [&]() {
                    wave_sync();   // staged keys visible to the wave
                    int64_t a0 = 0, a1 = 0;
                    if (lane < staged) { const int32_t b = wkb[wid][lane]; a0 = split[b]; a1 = off[b + 1]; }
                    nvis += (uint64_t)(a1 - a0);
                    uint64_t sw = 0;   // X(i,b) Wnt(i,j) <= d(i)^2 per entry
                    wave_walk_seg(a0, a1, wsa, wse, wsi[wid], [&](int64_t q) { return adj[q]; },
                                  [&](int y, int64_t, int32_t j) {
                                      const int32_t idx = j - gb;
                                      const uint32_t w = (ww[idx >> shift] >> ((idx & ((1 << shift) - 1)) * cb)) & cmask;
                                      sw += (uint64_t)wxs[wid][y] * w;
                                  });
                    part += sw;
                    staged = 0;   // the walk ends with a wave_sync: the arrays are free
                };
                for (int32_t kb = 0; kb < nk; kb += 64) {
                    const int32_t f = kb + lane;
                    uint32_t xv = 0;
                    if (f < nk) xv = (wx[f >> shift] >> ((f & ((1 << shift) - 1)) * cb)) & cmask;
                    const uint64_t m = __ballot(xv != 0);
                    if (m == 0) continue;
                    if (staged + __popcll(m) > 64) walk_staged();
                    if (xv) {
                        const int slot = staged + __popcll(m & lt);
                        wkb[wid][slot] = gb + f;
                        wxs[wid][slot] = xv;
                    }
                    staged += __popcll(m);
                }
                if (staged > 0) walk_staged();
                sc[0] += part;
                wave_sync();   // the tables are cleared by the wave's next source
            }
        }
        if (wgc >= 0) wave_flush_runs<1>(sc, wgc, acc, ACC_STRIDE, ids);
        flush_count(nvis, visits);
        return;
    }
    for (int q = threadIdx.x; q < 2 * slab; q += blockDim.x) dyn[q] = 0;
    if (threadIdx.x == 0) { s_nx = 0; s_nw = 0; }
    for (;;) {
        if (threadIdx.x == 0) s_i = slice_grab(task, slice_end);
        __syncthreads();
        const int gi = s_i;
        const int64_t t0 = task_begin(gi, chunk), tn = task_begin((int64_t)gi + 1, chunk);
        __syncthreads();   // s_i is read by every thread before it is taken again
        if (t0 >= n) {
            if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
            break;
        }
        const int32_t t1 = (int32_t)(tn < n ? tn : n);
        for (int32_t t = (int32_t)t0; t < t1; t++) {
        const int32_t i = n - 1 - t;
        const int g = gm.graph(i);
        block_switch_graph<1>(sc, gcur, g, red, acc, ACC_STRIDE, ids);
        // tables are indexed by rank relative to the start of i's graph
        const int32_t gb = gm.begin(g), ge = gm.end(g);
        const int32_t oi = off[i], si = split[i], ei = off[i + 1];
        // X(i,b) and Wnt(i,j) never exceed d(i): a low-degree source packs
        // several counts per word (count_shift), in LDS and in the tables
        const int shift = count_shift(ei - oi);
        const int cb = 32 >> shift;
        const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
        const int32_t hi0 = ge - (xslab << shift) > gb ? ge - (xslab << shift) : gb;   // first key held in LDS
        // count of key x in the LDS array s (latest keys) or the table t: add
        // one (returns the old count), read, clear; separate branches keep
        // LDS and global accesses apart
        auto inc = [&](uint32_t *s, uint32_t *t, int32_t x) -> uint32_t {
            const int32_t idx = x >= hi0 ? x - hi0 : x - gb;
            const uint32_t sh = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
            const uint32_t old = x >= hi0 ? atomicAdd(&s[idx >> shift], 1u << sh) : atomicAdd(&t[idx >> shift], 1u << sh);
            return (old >> sh) & cmask;
        };
        auto get = [&](const uint32_t *s, const uint32_t *t, int32_t x) -> uint32_t {
            const int32_t idx = x >= hi0 ? x - hi0 : x - gb;
            const uint32_t sh = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
            return ((x >= hi0 ? s[idx >> shift] : t[idx >> shift]) >> sh) & cmask;
        };
        auto clr = [&](uint32_t *s, uint32_t *t, int32_t x) {
            const int32_t idx = x >= hi0 ? x - hi0 : x - gb;
            const uint32_t sh = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
            // other counts of the word may be cleared concurrently
            if (x >= hi0) atomicAnd(&s[idx >> shift], ~(cmask << sh));
            else atomicAnd(&t[idx >> shift], ~(cmask << sh));
        };
        // X(i,b): a in N-(i), b in N+(a), b != i
        for (int32_t base = oi; base < si; base += blockDim.x) {
            int32_t p = base + threadIdx.x;
            int start = 0, len = 0;
            if (p < si) { int32_t a = adj[p]; start = split[a]; len = off[a + 1] - split[a]; }
            nvis += (uint64_t)len;
            lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                            [&](int, int64_t, int32_t b) {
                                if (b == i) return;
                                if (inc(sX, Xt, b) == 0) tx[atomicAdd(&s_nx, 1)] = b;
                            });
        }
        __syncthreads();
        if (s_nx == 0) continue;   // s_nw is still zero; the next write of s_nx is behind a barrier
        if (YSUM) {
            // The same sum taken from the other side: sum_j Wnt(i,j) Y(i,j)
            // with Y(i,j) = sum of X(i,b) over the keys b with j in N+(b).
            // The few out-rows of the keys b build Y (atomics); the many
            // Wnt wedges (c, j) only read it.  Y(i,j) < d(i) d(j) < 2^32
            // (maximum degree below 2^16): one word per key, LDS keys
            // [hy, ge), the rest in the workgroup's table, reset through
            // the touched list tw.
            const int32_t ys = 2 * slab - xslab;   // LDS words of the Y array
            const int32_t hy = ge - ys > gb ? ge - ys : gb;
            for (int q = threadIdx.x; q < ge - hy; q += blockDim.x) sW[q] = 0;
            __syncthreads();
            auto yadd = [&](int32_t j, uint32_t xv) {
                if (j >= hy) atomicAdd(&sW[j - hy], xv);
                else if (atomicAdd(&Wt[j - gb], xv) == 0) tw[atomicAdd(&s_nw, 1)] = j;   // xv >= 1
            };
            const int nx = s_nx;
            if (nx < FIVE_WAVE_KEYS) {
                for (int base = 0; base < nx; base += blockDim.x) {
                    const int xi = base + threadIdx.x;
                    int start = 0, len = 0;
                    if (xi < nx) { const int32_t b = tx[xi]; start = split[b]; len = off[b + 1] - split[b]; }
                    nvis += (uint64_t)len;
                    lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                                    [&](int s, int64_t, int32_t j) { yadd(j, get(sX, Xt, tx[base + s])); });
                }
            } else {
                const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
                int64_t *wsa = beg + wid * 64;
                int32_t *wse = pref + wid * 64;
                for (int xb = 0; xb < nx; xb += nwv * 64) {
                    const int xi = xb + lane * nwv + wid;   // keys dealt to the waves in turn
                    int64_t a0 = 0, a1 = 0;
                    uint32_t xv = 0;
                    if (xi < nx) {
                        const int32_t b = tx[xi];
                        a0 = split[b];
                        a1 = off[b + 1];
                        xv = get(sX, Xt, b);
                    }
                    nvis += (uint64_t)(a1 - a0);
                    wxs[wid][lane] = xv;   // visible to the wave after the walk's own wave_sync
                    wave_walk_seg(a0, a1, wsa, wse, wsi[wid], [&](int64_t q) { return adj[q]; },
                                  [&](int y, int64_t, int32_t j) { yadd(j, wxs[wid][y]); });
                }
            }
            __syncthreads();
            // Wnt wedges: c in N(i); all of N(c) when c is before i, else N+(c)
            uint64_t part = 0;
            for (int32_t base = oi; base < ei; base += blockDim.x) {
                int32_t p = base + threadIdx.x;
                int start = 0, len = 0;
                if (p < ei) {
                    int32_t cv = adj[p];
                    if (cv < i) { start = off[cv]; len = off[cv + 1] - off[cv]; }
                    else { start = split[cv]; len = off[cv + 1] - split[cv]; }
                }
                nvis += (uint64_t)len;
                lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                                [&](int, int64_t, int32_t j) {
                                    if (j == i) return;
                                    part += j >= hy ? sW[j - hy] : Wt[j - gb];
                                });
            }
            sc[0] += part;
            __syncthreads();
            for (int q = threadIdx.x; q < nx; q += blockDim.x) clr(sX, Xt, tx[q]);
            const int ny = s_nw;
            for (int q = threadIdx.x; q < ny; q += blockDim.x) Wt[tw[q] - gb] = 0;
            __syncthreads();
            if (threadIdx.x == 0) { s_nx = 0; s_nw = 0; }   // next reads are behind a barrier
            continue;
        }
        // Wnt(i,j): c in N(i); all of N(c) when c is before i, else only N+(c).
        // Its LDS keys are only read afterwards, never listed: the array is
        // cleared here and counted without return values; table keys are
        // listed for their reset.
        {
            const int32_t swn = ((ge - hi0) + (1 << shift) - 1) >> shift;   // words holding keys [hi0, ge)
            for (int q = threadIdx.x; q < swn; q += blockDim.x) sW[q] = 0;
            __syncthreads();
        }
        for (int32_t base = oi; base < ei; base += blockDim.x) {
            int32_t p = base + threadIdx.x;
            int start = 0, len = 0;
            if (p < ei) {
                int32_t cv = adj[p];
                if (cv < i) { start = off[cv]; len = off[cv + 1] - off[cv]; }
                else { start = split[cv]; len = off[cv + 1] - split[cv]; }
            }
            lbs_batch(start, len, pref, beg, tmp, [&](int, int q) {
                int32_t j = adj[q];
                nvis++;
                if (j == i) return;
                if (j >= hi0) {
                    const int32_t idx = j - hi0;
                    atomicAdd(&sW[idx >> shift], 1u << ((idx & ((1 << shift) - 1)) * cb));
                } else if (inc(sW, Wt, j) == 0) {
                    tw[atomicAdd(&s_nw, 1)] = j;
                }
            });
        }
        __syncthreads();
        // sum_b X(i,b) sum_{j in N+(b)} Wnt(i,j).  With enough keys b they are
        // dealt to the waves in turn and each wave walks the out-rows of its
        // 64 as one flattened run; with few, the block shares their elements
        // (lbs_batch)
        const int nx = s_nx;
        if (!WALK || nx < FIVE_WAVE_KEYS) {
            for (int base = 0; base < nx; base += blockDim.x) {
                const int xi = base + threadIdx.x;
                int start = 0, len = 0;
                if (xi < nx) { const int32_t b = tx[xi]; start = split[b]; len = off[b + 1] - split[b]; }
                nvis += (uint64_t)len;
                lbs_batch(start, len, pref, beg, tmp, [&](int s, int q) {
                    const int32_t b = tx[base + s];
                    sc[0] += (uint64_t)get(sX, Xt, b) * get(sW, Wt, adj[q]);
                });
            }
        } else {
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
            int64_t *wsa = beg + wid * 64;
            int32_t *wse = pref + wid * 64;
            for (int xb = 0; xb < nx; xb += nwv * 64) {
                const int xi = xb + lane * nwv + wid;   // keys dealt to the waves in turn
                int64_t a0 = 0, a1 = 0;
                uint32_t xv = 0;
                if (xi < nx) {
                    const int32_t b = tx[xi];
                    a0 = split[b];
                    a1 = off[b + 1];
                    xv = get(sX, Xt, b);
                }
                nvis += (uint64_t)(a1 - a0);
                wxs[wid][lane] = xv;   // visible to the wave after the walk's own wave_sync
                wave_walk_seg(a0, a1, wsa, wse, wsi[wid], [&](int64_t q) { return adj[q]; },
                              [&](int y, int64_t, int32_t j) { sc[0] += (uint64_t)wxs[wid][y] * get(sW, Wt, j); });
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nx; q += blockDim.x) {
            const int32_t b = tx[q];
            clr(sX, Xt, b);
        }
        const int nw = s_nw;
        for (int q = threadIdx.x; q < nw; q += blockDim.x) {
            const int32_t j = tw[q];
            clr(sW, Wt, j);
        }
        __syncthreads();
        if (threadIdx.x == 0) { s_nx = 0; s_nw = 0; }   // next reads are behind a barrier
        }
    }
    if (gcur >= 0) block_flush_u128<1>(sc, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    flush_count(nvis, visits);
}


// -------------------------------------------------- pattern 17, hub pairs
//
// Nearly all diamond work of a heavy-tailed graph has both tips among the
// latest ranks (the hubs): an edge (k,l) inside the common neighbourhood of
// many hubs is met once per pair of them.  Let the hubs be the latest R ranks
// and call an edge dense when at least Q hubs are apexes of its triangles.
// For hub tips i < j, the dense edges inside N(i) & N(j) number
//     Dd(i,j) = sum_e Y(i,e) Y(j,e),   Y(v,e) = 1 when v is an apex of e,
// a dense contraction over the dense edges.  The pattern-17 sum splits as
// the diamond walk over the edges that are not dense (hub sources skip the
// dense ones) plus sum_{hub i < j} (W(i,j) - 2) Dd(i,j), W from the rows
// the hub sources keep.  Y is built in chunks of HUB_EC dense edges (4-bit
// entries, 0 or 1.0) and contracted on the matrix cores (tiles.h): the 0/1
// entries multiply exactly and a chunk's counts stay below 2^24.

#define HUB_EC 131072  // dense edges per chunk of Y (two to a byte of a Y row)

// Dense arcs of each row k: the arcs k -> l (l after k) whose triangle lists
// hold at least q apexes from hub0 on (the lists are sorted by apex).  A
// wave per row; cnt[k] = number of dense arcs.
template <bool IDS>
__global__ void __launch_bounds__(256) k_hub_count(int32_t n, const int32_t *off, const int32_t *split,
                                                   const int32_t *adj, const int64_t *aoff, const uint32_t *aa,
                                                   const int32_t *av, int32_t hub0, int32_t qmin, int64_t *cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k = w0; k < n; k += nwv) {
        uint32_t c = 0;
        for (int32_t q = split[k] + lane; q < off[k + 1]; q += 64) {
            int64_t lo = aoff[q], hi = aoff[q + 1];
            const int64_t end = hi;
            while (lo < hi) { const int64_t mid = (lo + hi) >> 1; if (apex_at<IDS>(av, adj, aa, mid) < hub0) lo = mid + 1; else hi = mid; }
            c += end - lo >= qmin;
        }
        c = (uint32_t)wave_sum_u64(c);
        if (lane == 0) cnt[k] = c;
    }
}

// Number the dense arcs in arc order from base[k] (did = -1 for the other
// arcs after the split); chunk c of HUB_EC numbers spans rows
// kr[2c] .. kr[2c+1].
template <bool IDS>
__global__ void __launch_bounds__(256) k_hub_number(int32_t n, const int32_t *off, const int32_t *split,
                                                    const int32_t *adj, const int64_t *aoff, const uint32_t *aa,
                                                    const int32_t *av, int32_t hub0, int32_t qmin,
                                                    const int64_t *base, int32_t *did, int32_t *kr) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t total = base[n];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t k = w0; k < n; k += nwv) {
        int64_t next = base[k];
        for (int32_t qb = split[k]; qb < off[k + 1]; qb += 64) {
            const int32_t q = qb + lane;
            bool dense = false;
            if (q < off[k + 1]) {
                int64_t lo = aoff[q], hi = aoff[q + 1];
                const int64_t end = hi;
                while (lo < hi) { const int64_t mid = (lo + hi) >> 1; if (apex_at<IDS>(av, adj, aa, mid) < hub0) lo = mid + 1; else hi = mid; }
                dense = end - lo >= qmin;
            }
            const uint64_t m = __ballot(dense);
            if (q < off[k + 1]) {
                const int64_t d = next + __popcll(m & below);
                did[q] = dense ? (int32_t)d : -1;
                if (dense) {
                    if (d % HUB_EC == 0) kr[2 * (d / HUB_EC)] = (int32_t)k;
                    if (d % HUB_EC == HUB_EC - 1 || d == total - 1) kr[2 * (d / HUB_EC) + 1] = (int32_t)k;
                }
            }
            next += __popcll(m);
        }
    }
}

// Rows of Y for one chunk: a workgroup per hub i sets, in an LDS row of kb
// bytes, the entry of every dense edge (k,l) of the chunk with i as apex --
// the entries l after k of the lists of the arcs (i,k), k in the chunk's
// rows -- then stores the row.
template <bool IDS>
__global__ void __launch_bounds__(256) k_hub_rows(const int32_t *off, const int32_t *adj, const int32_t *rev,
                                                  const int64_t *aoff, const uint32_t *aa, const int32_t *av,
                                                  int32_t hub0, const int32_t *did, int64_t base, int32_t kb,
                                                  const int32_t *kr, int32_t chunk, uint8_t *y) {
    extern __shared__ uint32_t rowb[];
    __shared__ int pref[257], tmp[8];
    __shared__ int64_t beg[257];
    const int32_t i = hub0 + (int32_t)blockIdx.x;
    for (int q = threadIdx.x; q < kb / 4; q += blockDim.x) rowb[q] = 0;
    const int32_t kf = kr[2 * chunk], kl = kr[2 * chunk + 1];
    int32_t p0 = off[i], p1 = off[i + 1];
    {
        int32_t lo = p0, hi = p1;
        while (lo < hi) { const int32_t mid = (lo + hi) >> 1; if (adj[mid] < kf) lo = mid + 1; else hi = mid; }
        p0 = lo;
        hi = p1;
        while (lo < hi) { const int32_t mid = (lo + hi) >> 1; if (adj[mid] <= kl) lo = mid + 1; else hi = mid; }
        p1 = lo;
    }
    __syncthreads();
    for (int32_t bp = p0; bp < p1; bp += blockDim.x) {
        const int32_t p = bp + threadIdx.x;
        int64_t start = 0;
        int len = 0;
        if (p < p1) { start = aoff[p]; len = (int)(aoff[p + 1] - start); }
        lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t x) { return aa[x]; },
                        [&](int s, int64_t x, uint32_t ax) {
            const int32_t pk = bp + s;
            if (ax > (uint32_t)pk) {   // l > k: the arc (i,l) after (i,k) in row i
                const int32_t qkl = (int32_t)aa[aoff[rev[pk]] + (x - beg[s])];   // arc (k,l) in row k
                const int64_t e = (int64_t)did[qkl] - base;
                if (did[qkl] >= 0 && e >= 0 && e < 2 * (int64_t)kb) fp4_set_one(rowb, e);
            }
        });
    }
    __syncthreads();
    uint4 *dst = (uint4 *)(y + (size_t)blockIdx.x * kb);
    const uint4 *src = (const uint4 *)rowb;
    for (int q = threadIdx.x; q < kb / 16; q += blockDim.x) dst[q] = src[q];
}

// sum over hub pairs i < j of one tile of (W(i,j) - 2) sum_e Y(i,e) Y(j,e),
// over the kb bytes of the chunk's rows (tiles by patch, see above)
__global__ void __launch_bounds__(64 * HUB_WAVES) k_hub_gemm(const uint8_t *y, int32_t hub_r, int32_t kb, const void *wtop,
                                                  int w16, int32_t nb, unsigned long long *acc) {
    extern __shared__ __attribute__((aligned(16))) uint8_t hub_lds[];
    __shared__ u128 red[HUB_WAVES];
    const int local = (int)(blockIdx.x >> 3), xcd = (int)(blockIdx.x & 7);
    int ti, tj;
    if (!hub_patch_tile(nb, (local / (HUB_PR * HUB_PC)) * 8 + xcd, local % (HUB_PR * HUB_PC), &ti, &tj))
        return;   // the whole workgroup leaves
    hub_v4f cacc[8][HUB_BC];
    hub_tile((lds_u8 *)hub_lds, y, kb, ti, tj, cacc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t s = 0;
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < HUB_BC; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int32_t i = ti * HUB_T + hub_acc_row(wid, lane, a, r);
                const int32_t j = tj * HUB_T + hub_acc_col(wid, lane, b);
                if (i < j) {
                    const size_t wi = (size_t)i * hub_r + j;
                    const uint32_t w = w16 ? ((const uint16_t *)wtop)[wi] : ((const uint32_t *)wtop)[wi];
                    // a row left at 0 belongs to a source of degree <= 2, whose
                    // pairs with a common edge have W = 2
                    if (w > 2) s += (uint64_t)(w - 2) * (uint32_t)cacc[a][b][r];   // exact integer count
                }
            }
    u128 v[1] = {(u128)s};
    const int ids[1] = {AC_N17};
    block_flush_u128<1>(v, red, acc, ids);
}

// ------------------------------------------------ pattern 18, dense hubs
//
// The rim 4-cycles of a hub h are the 4-cycles of G[N(h)]: with A_h its
// 0/1 adjacency (rows and columns the positions in the row of h) and
// c(i,j) = (A_h A_h)(i,j) the common neighbours of rim vertices i, j inside
// N(h), each 4-cycle has two diagonals, so the hub's count is
// (1/2) sum_{i<j} C(c(i,j), 2).  A hub whose walk would visit many list
// entries (about S2/4, S2 = sum over its arcs of t^2) for its d^3/2
// multiply-adds takes this product on the matrix cores (tiles.h); the sum is
// gathered twice over in AC_WD2 and halved when the counts are combined.
// A batch of such hubs: matrix of hub q at byte mo[q] (dpad[q] x dpad[q],
// dpad = d rounded up to HUB_T, zero beyond d), rows numbered from rp[q],
// patches of its tile grid from pp[q].

// row i of hub q's matrix: the list of arc (h, i-th neighbour) holds the
// positions of the common neighbours in the row of h
__global__ void __launch_bounds__(256) k_wheel_rows(const int32_t *off, const int64_t *aoff, const uint32_t *aa,
                                                    int32_t nh, const int32_t *hub, const int32_t *dpad,
                                                    const int64_t *rp, const int64_t *mo, uint8_t *y) {
    extern __shared__ uint32_t rowb[];
    int lo = 0, hi = nh - 1;   // last hub whose first row is <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const int32_t h = hub[lo], dp = dpad[lo], rb = dp / 2;   // row bytes: two entries each
    const int64_t i = (int64_t)blockIdx.x - rp[lo];
    const int32_t oh = off[h], d = off[h + 1] - oh;
    for (int q = threadIdx.x; q < rb / 4; q += blockDim.x) rowb[q] = 0;
    __syncthreads();
    if (i < d) {
        const int64_t x0 = aoff[oh + i], x1 = aoff[oh + i + 1];
        for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) fp4_set_one(rowb, (int32_t)aa[x] - oh);
    }
    __syncthreads();
    uint4 *dst = (uint4 *)(y + mo[lo] + i * (int64_t)rb);
    const uint4 *src = (const uint4 *)rowb;
    for (int q = threadIdx.x; q < rb / 16; q += blockDim.x) dst[q] = src[q];
}

// sum over the hubs of a batch and their rim pairs i < j of C(c(i,j), 2)
__global__ void __launch_bounds__(64 * HUB_WAVES) k_wheel_gemm(const uint8_t *y, int32_t nh, const int32_t *dpad,
                                                    const int64_t *mo, const int32_t *pp,
                                                    unsigned long long *acc) {
    extern __shared__ __attribute__((aligned(16))) uint8_t hub_lds[];
    __shared__ u128 red[HUB_WAVES];
    const int local = (int)(blockIdx.x >> 3), xcd = (int)(blockIdx.x & 7);
    const int P = (local / (HUB_PR * HUB_PC)) * 8 + xcd;
    if (P >= pp[nh]) return;   // the whole workgroup leaves
    int lo = 0, hi = nh - 1;   // hub of patch P
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pp[mid] <= P) lo = mid; else hi = mid - 1;
    }
    const int32_t dp = dpad[lo];
    int ti, tj;
    if (!hub_patch_tile(dp / HUB_T, P - pp[lo], local % (HUB_PR * HUB_PC), &ti, &tj)) return;
    hub_v4f cacc[8][HUB_BC];
    hub_tile((lds_u8 *)hub_lds, y + mo[lo], dp / 2, ti, tj, cacc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t s = 0;
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < HUB_BC; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int32_t i = ti * HUB_T + hub_acc_row(wid, lane, a, r);
                const int32_t j = tj * HUB_T + hub_acc_col(wid, lane, b);
                const uint64_t cij = (uint32_t)cacc[a][b][r];   // exact: an integer below 2^17
                if (i < j) s += cij * (cij - (cij > 0)) / 2;
            }
    u128 v[1] = {(u128)s};
    const int ids[1] = {AC_WD2};
    block_flush_u128<1>(v, red, acc, ids);
}

// S2 = sum over the arcs of hub h of t^2, for the candidates from rank lo on
// (a wave per hub)
__global__ void __launch_bounds__(256) k_wheel_s2(int32_t lo, int32_t n, const int32_t *off, const uint32_t *tarc,
                                                  unsigned long long *s2) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t h = lo + w0; h < n; h += nwv) {
        uint64_t x = 0;
        for (int32_t p = off[h] + lane; p < off[h + 1]; p += 64) x += (uint64_t)tarc[p] * tarc[p];
        x = wave_sum_u64(x);
        if (lane == 0) s2[h - lo] = x;
    }
}

// ------------------------------------------------------------------- stages

static esc_status pair_scratch(esc_ctx *c, uint32_t **tab, int32_t **touch, int **task) {
    size_t per = (size_t)c->tab_n * sizeof(uint32_t);
    int nwg = pair_wgs(c);
    *tab = (uint32_t *)ctx_buf(c, B_WG_SCRATCH, per * 2 * nwg);
    *touch = (int32_t *)ctx_buf(c, B_WG_TOUCH, per * 2 * nwg);
    *task = (int *)ctx_buf(c, B_TASK, sizeof(int) * 16);
    if (!*tab || !*touch || !*task) return ESC_ENOMEM;
    return ESC_OK;
}

// The hub-pair split of pattern 17 (above) for one graph: numbers the dense
// edges and clears the kept W rows.  *hub0 = the first hub rank, or n when
// the split is off (a batch, too few vertices, no memory); *ndense = the
// number of dense edges.
static esc_status hub_prepare(esc_ctx *c, int32_t *hub0, int64_t *ndense) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    // -1: about one rank in 160, in whole tiles, at most 24576
    int32_t R = c->pairs_hub_r;
    if (R < 0) {
        R = (int32_t)(((int64_t)n / 160) / HUB_T * HUB_T);
        if (R > 24576) R = 24576;
    }
    *hub0 = n;
    *ndense = 0;
    if (c->G || R <= 0 || (int64_t)n < 2 * (int64_t)R || c->narcs_apex == 0) return ESC_OK;
    // the product's operand tiles and a chunk's Y row must fit a workgroup's LDS
    if ((size_t)c->max_lds < 4 * (size_t)HUB_T * HUB_K + 1024 || (size_t)c->max_lds < (size_t)HUB_EC / 2 + 4096)
        return ESC_OK;
    // memory: what the buffers need beyond what they already hold, with 1 GiB
    // left over for the later stages
    const Buf bufs[6] = {B_HUB_DID, B_HUB_CNT, B_HUB_BASE, B_HUB_KR, B_HUB_W, B_HUB_Y};
    const size_t sizes[6] = {sizeof(int32_t) * (size_t)c->m2, sizeof(int64_t) * (size_t)(n + 1),
                             sizeof(int64_t) * (size_t)(n + 1), sizeof(int32_t) * 2 * (size_t)(c->m / HUB_EC + 2),
                             (c->maxdeg < 65536 ? 2 : 4) * (size_t)R * R, (size_t)R * HUB_EC / 2};
    size_t more = 0;
    for (int b = 0; b < 6; b++) {
        const size_t want = sizes[b] + sizes[b] / 8 + ((size_t)2 << 20);   // ctx_buf's rounding
        if (ctx_held(c, bufs[b]) < sizes[b]) more += want - ctx_held(c, bufs[b]);
    }
    size_t free_b = 0;
    ESC_TRY(ctx_free_bytes(c, &free_b));
    if (more + ((size_t)1 << 30) > free_b) return ESC_OK;
    if (c->budget && c->held + more > c->budget) return ESC_OK;
    int32_t *did = (int32_t *)ctx_buf(c, B_HUB_DID, sizeof(int32_t) * (size_t)c->m2);
    int64_t *cnt = (int64_t *)ctx_buf(c, B_HUB_CNT, sizeof(int64_t) * (size_t)(n + 1));
    int64_t *base = (int64_t *)ctx_buf(c, B_HUB_BASE, sizeof(int64_t) * (size_t)(n + 1));
    int32_t *kr = (int32_t *)ctx_buf(c, B_HUB_KR, sizeof(int32_t) * 2 * (size_t)(c->m / HUB_EC + 2));
    // W(i,j) <= d(i): 16-bit entries when every degree is below 2^16
    c->hub_w16 = c->maxdeg < 65536;
    const size_t wbytes = (c->hub_w16 ? 2 : 4) * (size_t)R * R;
    void *wtop = ctx_buf(c, B_HUB_W, wbytes);
    uint8_t *y = (uint8_t *)ctx_buf(c, B_HUB_Y, (size_t)R * HUB_EC / 2);
    if (!did || !cnt || !base || !kr || !wtop || !y) return ESC_OK;   // no room after all: off
    c->pairs_hub_used = R;
    const int32_t h0 = n - R;
    const int grid = grid_cap(c, (int64_t)n * 64, 256);
    const int32_t *off = (const int32_t *)c->buf[B_OFF], *split = (const int32_t *)c->buf[B_SPLIT];
    const int32_t *adj = (const int32_t *)c->buf[B_ADJ];
    const int64_t *aoff = (const int64_t *)c->buf[B_AOFF];
    const uint32_t *aa = (const uint32_t *)c->buf[B_AA];
    HIP_TRY(hipMemsetAsync(cnt + n, 0, sizeof(int64_t), st));
    if (c->av) k_hub_count<true><<<grid, 256, 0, st>>>(n, off, split, adj, aoff, aa, c->av, h0, c->pairs_hub_q, cnt);
    else k_hub_count<false><<<grid, 256, 0, st>>>(n, off, split, adj, aoff, aa, c->av, h0, c->pairs_hub_q, cnt);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, cnt, base, n + 1));
    if (c->av) k_hub_number<true><<<grid, 256, 0, st>>>(n, off, split, adj, aoff, aa, c->av, h0, c->pairs_hub_q, base, did, kr);
    else k_hub_number<false><<<grid, 256, 0, st>>>(n, off, split, adj, aoff, aa, c->av, h0, c->pairs_hub_q, base, did, kr);
    HIP_TRY(hipGetLastError());
    int64_t nd = 0;
    HIP_TRY(hipMemcpyAsync(&nd, base + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemsetAsync(wtop, 0, wbytes, st));
    HIP_TRY(hipStreamSynchronize(st));
    *hub0 = h0;
    *ndense = nd;
    return ESC_OK;
}

// sum_{hub i < j} (W(i,j) - 2) Dd(i,j) into pattern 17, chunk by chunk of
// the dense edges
static esc_status hub_product(esc_ctx *c, int32_t hub0, int64_t ndense) {
    const int32_t R = c->pairs_hub_used;
    hipStream_t st = c->stream;
    if (ndense == 0) return ESC_OK;
    uint8_t *y = (uint8_t *)c->buf[B_HUB_Y];
    const int32_t nb = R / HUB_T;
    const int nwg = 8 * HUB_PR * HUB_PC * ((hub_npatches(nb) + 7) / 8);
    const size_t lds = 4 * (size_t)HUB_T * HUB_K;   // two buffers of both operands
    const int64_t nchunks = (ndense + HUB_EC - 1) / HUB_EC;
    auto rows = c->av ? k_hub_rows<true> : k_hub_rows<false>;
    for (int64_t ch = 0; ch < nchunks; ch++) {
        const int64_t base = ch * HUB_EC;
        const int64_t left = ndense - base < HUB_EC ? ndense - base : HUB_EC;
        const int32_t kb = (int32_t)(((left + 1) / 2 + HUB_K - 1) / HUB_K * HUB_K);   // bytes: two entries each
        rows<<<R, 256, (size_t)kb, st>>>((const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ],
                                         (const int32_t *)c->buf[B_REV], (const int64_t *)c->buf[B_AOFF],
                                         (const uint32_t *)c->buf[B_AA], c->av, hub0,
                                         (const int32_t *)c->buf[B_HUB_DID], base, kb,
                                         (const int32_t *)c->buf[B_HUB_KR], (int32_t)ch, y);
        HIP_TRY(hipGetLastError());
        k_hub_gemm<<<nwg, 64 * HUB_WAVES, lds, st>>>(y, R, kb, c->buf[B_HUB_W], c->hub_w16 ? 1 : 0, nb,
                                          (unsigned long long *)c->buf[B_ACC]);
        HIP_TRY(hipGetLastError());
        c->prod_macs[STAGE_PAIRS] += (uint64_t)(nb * (nb + 1) / 2) * HUB_T * HUB_T * 2 * (uint64_t)kb;
    }
    return ESC_OK;
}

esc_status stage_pairs(esc_ctx *c) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    if (n == 0 || c->m == 0) return ESC_OK;   // no wedge: nothing to add, no tables to size
    uint32_t *tab;
    int32_t *touch;
    int *task;
    ESC_TRY(pair_scratch(c, &tab, &touch, &task));
    int32_t hub0 = n;
    int64_t ndense = 0;
    c->pairs_hub_used = 0;
    ESC_TRY(hub_prepare(c, &hub0, &ndense));
    HIP_TRY(hipMemsetAsync(task, 0, sizeof(int) * 16, st));
    // LDS slab for the latest keys of a graph, leaving room for the static arrays
    const int32_t slab = slab_words(c, slab_wgs_per_cu(c), 1, 16384, 16384);
    // a batch whose graphs are small takes a source per wave, with per-wave
    // LDS tables over a graph's keys (16-bit counts at most); its diamond
    // suffixes are staged as start << 24 | length (lists below 2^40 entries)
    const int32_t pw_words = c->G && c->tab_n <= 4096 && c->narcs_apex < ((int64_t)1 << 40) ? (c->tab_n + 1) / 2 : 0;
    const int32_t lds_words = 8 * pw_words > slab ? 8 * pw_words : (slab > 0 ? slab : 1);
    auto kern = c->av ? k_pairs_wd<true> : k_pairs_wd<false>;
    const int32_t *did = hub0 < n ? (const int32_t *)c->buf[B_HUB_DID] : nullptr;
    void *wtop = hub0 < n ? c->buf[B_HUB_W] : nullptr;
    ESC_TRY(run_sliced(c, "pairs_13_17", task + 8, task, [&](uint64_t ticks) -> esc_status {
        kern<<<slab_wgs_per_cu(c) * c->num_cu, 512, sizeof(uint32_t) * (size_t)lds_words, st>>>(
            n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_REV],
            (const int64_t *)c->buf[B_AOFF], (const uint32_t *)c->buf[B_AA], c->av, tab, touch, c->tab_n,
            c->task_chunk, gmap_of(c), task, slab, pw_words, (unsigned long long *)c->buf[B_ACC],
            (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 6, ticks, task + 8, hub0, c->pairs_hub_used, did, wtop,
            c->hub_w16 ? 1 : 0);
        HIP_TRY(hipGetLastError());
        return ESC_OK;
    }));
    ESC_TRY(mark_walk_end(c, STAGE_PAIRS));
    if (hub0 < n) ESC_TRY(hub_product(c, hub0, ndense));
    return ctx_release_if_short(c, {B_HUB_Y, B_HUB_W, B_HUB_DID});
}

#define WD_CAND 65536      // hubs (latest ranks) considered for the dense wheel product
#define WD_MAX_DEG 65536   // and at most this degree (its matrix row in LDS, 4 GiB matrix)

// Hubs of one graph whose wheels go to the product: degree at least
// wheel_dense_deg (and at most WD_MAX_DEG), among the latest WD_CAND ranks,
// with dpad^3 / 2 < wheel_dense_ratio * S2 / 4.  *wd_lo = first candidate
// rank, B_WD_FLAG[h - wd_lo] = 1 for the chosen hubs (listed in *dense).
static esc_status wheel_dense_select(esc_ctx *c, int32_t *wd_lo, std::vector<int32_t> *dense) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    *wd_lo = n;
    if (c->G || c->wheel_dense_deg <= 0 || c->maxdeg < c->wheel_dense_deg) return ESC_OK;
    if ((size_t)c->max_lds < 4 * (size_t)HUB_T * HUB_K + 1024) return ESC_OK;
    // S2 of the latest K ranks and their row offsets, read back together
    const int32_t K = n < WD_CAND ? n : WD_CAND;
    unsigned long long *s2 = (unsigned long long *)ctx_buf(c, B_WD_S2, sizeof(uint64_t) * (size_t)K);
    uint8_t *flag = (uint8_t *)ctx_buf(c, B_WD_FLAG, (size_t)K);
    if (!s2 || !flag) return ESC_ENOMEM;
    k_wheel_s2<<<grid_cap(c, (int64_t)K * 64, 256), 256, 0, st>>>(n - K, n, (const int32_t *)c->buf[B_OFF],
                                                                  (const uint32_t *)c->buf[B_TARC], s2);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> &hoff = c->wd_degs;
    hoff.resize((size_t)K + 1);
    std::vector<uint64_t> hs2((size_t)K);
    HIP_TRY(hipMemcpyAsync(hoff.data(), (const int32_t *)c->buf[B_OFF] + (n - K), sizeof(int32_t) * ((size_t)K + 1),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hs2.data(), s2, sizeof(uint64_t) * (size_t)K, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->wd_base = n - K;
    int32_t first = K;   // first of the latest K ranks with degree >= wheel_dense_deg (degrees ascend)
    while (first > 0 && hoff[first] - hoff[first - 1] >= c->wheel_dense_deg) first--;
    if (first == K) return ESC_OK;
    // matrix buffer: every chosen matrix, at most 8 GiB (the hubs then go in
    // batches), at least the largest one; a matrix larger than the memory
    // the buffer can have leaves its hub to the walk
    size_t free_b = 0;
    ESC_TRY(ctx_free_bytes(c, &free_b));
    const size_t room = ctx_held(c, B_WD_Y) + (free_b > ((size_t)2 << 30) ? (free_b - ((size_t)2 << 30)) / 2 : 0);
    std::vector<uint8_t> &hf = c->wd_flags;   // kept until the next call: the copy below reads it
    hf.assign((size_t)K, 0);
    size_t total = 0, biggest = 0;
    for (int32_t q = first; q < K; q++) {
        const int32_t h = n - K + q;
        const int64_t d = hoff[q + 1] - hoff[q];
        if (d > WD_MAX_DEG) continue;
        const int64_t dpi = (d + HUB_T - 1) / HUB_T * HUB_T;
        const double dp = (double)dpi;
        const size_t mbytes = (size_t)(dpi * dpi / 2);   // two entries a byte
        if (mbytes > room) continue;
        if (dp * dp * dp / 2 < (double)c->wheel_dense_ratio * (double)hs2[q] / 4) {
            hf[q] = 1;
            dense->push_back(h);
            total += mbytes;
            biggest = mbytes > biggest ? mbytes : biggest;
        }
    }
    if (dense->empty()) return ESC_OK;
    size_t cap = total < ((size_t)8 << 30) ? total : ((size_t)8 << 30);
    if (cap < biggest) cap = biggest;
    if (cap > room) cap = room;   // >= biggest: every chosen matrix fits the room
    c->wd_cap = cap;
    HIP_TRY(hipMemcpyAsync(flag, hf.data(), (size_t)K, hipMemcpyHostToDevice, st));
    *wd_lo = n - K;
    return ESC_OK;
}

// The chosen hubs in batches whose matrices fit the buffer: rows, then the
// tile products of every hub of the batch in one launch.
static esc_status wheel_dense_product(esc_ctx *c, const std::vector<int32_t> &dense) {
    if (dense.empty()) return ESC_OK;
    hipStream_t st = c->stream;
    const int32_t n = c->n, K = n < WD_CAND ? n : WD_CAND;
    auto deg = [&](int32_t h) { return (int64_t)(c->wd_degs[h - c->wd_base + 1] - c->wd_degs[h - c->wd_base]); };
    auto pad = [&](int32_t h) { return (deg(h) + HUB_T - 1) / HUB_T * HUB_T; };
    (void)K;
    const size_t cap = c->wd_cap;   // holds the largest chosen matrix (wheel_dense_select)
    uint8_t *y = (uint8_t *)ctx_buf(c, B_WD_Y, cap);
    // per batch: hub, dpad, first row, matrix offset, first patch (int64 each)
    const size_t nd = dense.size();
    int64_t *meta = (int64_t *)ctx_buf(c, B_WD_META, sizeof(int64_t) * 5 * (nd + 1));
    if (!y || !meta) return ESC_ENOMEM;
    std::vector<int32_t> hub(nd + 1), dp(nd + 1), pp(nd + 1);
    std::vector<int64_t> rp(nd + 1), mo(nd + 1);
    const size_t lds = 4 * (size_t)HUB_T * HUB_K;
    size_t q0 = 0;
    while (q0 < nd) {
        // one batch: hubs q0 .. q1-1
        size_t q1 = q0;
        int64_t bytes = 0, rows = 0;
        int32_t patches = 0, maxdp = 0;
        while (q1 < nd) {
            const int64_t p = pad(dense[q1]);
            if (q1 > q0 && bytes + p * p / 2 > (int64_t)cap) break;
            hub[q1 - q0] = dense[q1];
            dp[q1 - q0] = (int32_t)p;
            rp[q1 - q0] = rows;
            mo[q1 - q0] = bytes;
            pp[q1 - q0] = patches;
            rows += p;
            bytes += p * p / 2;
            patches += hub_npatches((int)(p / HUB_T));
            maxdp = (int32_t)p > maxdp ? (int32_t)p : maxdp;
            c->prod_macs[STAGE_WHEELS] += (uint64_t)((p / HUB_T) * (p / HUB_T + 1) / 2) * HUB_T * HUB_T * (uint64_t)p;
            q1++;
        }
        const int32_t nh = (int32_t)(q1 - q0);
        rp[nh] = rows;
        mo[nh] = bytes;
        pp[nh] = patches;
        int32_t *d_hub = (int32_t *)meta, *d_dp = d_hub + (nd + 1), *d_pp = d_dp + (nd + 1);
        int64_t *d_rp = (int64_t *)(d_pp + (nd + 1) + ((nd + 1) & 1)), *d_mo = d_rp + (nd + 1);
        HIP_TRY(hipMemcpyAsync(d_hub, hub.data(), sizeof(int32_t) * (nh + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_dp, dp.data(), sizeof(int32_t) * (nh + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_pp, pp.data(), sizeof(int32_t) * (nh + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_rp, rp.data(), sizeof(int64_t) * (nh + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_mo, mo.data(), sizeof(int64_t) * (nh + 1), hipMemcpyHostToDevice, st));
        k_wheel_rows<<<(unsigned)rows, 256, (size_t)maxdp / 2, st>>>((const int32_t *)c->buf[B_OFF],
                                                                (const int64_t *)c->buf[B_AOFF],
                                                                (const uint32_t *)c->buf[B_AA], nh, d_hub, d_dp, d_rp,
                                                                d_mo, y);
        HIP_TRY(hipGetLastError());
        const int nwg = 8 * HUB_PR * HUB_PC * ((patches + 7) / 8);
        k_wheel_gemm<<<nwg, 64 * HUB_WAVES, lds, st>>>(y, nh, d_dp, d_mo, d_pp, (unsigned long long *)c->buf[B_ACC]);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));   // the host arrays are rewritten by the next batch
        q0 = q1;
    }
    return ESC_OK;
}

esc_status stage_wheels(esc_ctx *c) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    if (n == 0 || c->narcs_apex == 0) return ESC_OK;
    // eight waves per workgroup for one graph; four for a batch of small
    // graphs, whose hubs have few rim vertices to share among the waves
    const int waves = c->G ? 4 : WHEEL_WAVES;
    // The kernel holds four waves per SIMD (its registers), so two 8-wave
    // workgroups per CU: each gets half the CU's LDS less its static arrays
    // (10 KB) for its tables.  Large-hub tasks: wk 16-bit counts (a range
    // of keys); per-wave mode: a table and a touched list of (wq + 1) / 2
    // words each per wave, wq the largest hub it takes.
    const int32_t budget = (int32_t)(((size_t)c->max_lds / 2 - 12288) / 4) & ~63;   // words
    const int32_t wk = 2 * budget;    // keys per range of a large-hub task
    // per-wave mode up to a hub of wq neighbours: an eighth (a quarter for
    // batches) of the keys the largest hub has, so graphs with small hubs
    // keep small tables and more workgroups per CU
    int32_t cap = c->maxdeg + 1 < wk ? c->maxdeg + 1 : wk;
    int32_t wq = cap / waves;
    if (wq > budget / waves) wq = budget / waves;
    const int32_t tab_words = (cap + 1) / 2;   // a large-hub task's table
    const int32_t wave_words_all = waves * 2 * ((wq + 1) / 2);
    size_t lds = sizeof(uint32_t) * (size_t)(tab_words > wave_words_all ? tab_words : wave_words_all);
    // hubs of at most WHEEL_TINY neighbours are taken whole, one per wave,
    // in the wave's one-wave table when it holds WHEEL_TINY_WORDS words,
    // else in tables after those (a batch of small graphs)
    const int tiny = WHEEL_TINY;
    if (2 * ((wq + 1) / 2) < WHEEL_TINY_WORDS) lds += sizeof(uint32_t) * waves * (size_t)WHEEL_TINY_WORDS;
    int per_cu = (int)(c->max_lds / (lds + 10240));
    if (per_cu > 4) per_cu = 4;
    if (per_cu < 1) per_cu = 1;
    int *task = (int *)ctx_buf(c, B_TASK, sizeof(int) * 16);
    // hubs counted by the product instead of the walk
    int32_t wd_lo = n;
    std::vector<int32_t> dense;
    ESC_TRY(wheel_dense_select(c, &wd_lo, &dense));
    const uint8_t *wflag = wd_lo < n ? (const uint8_t *)c->buf[B_WD_FLAG] : nullptr;
    // tasks of the hubs with more than wq neighbours
    int64_t *len = (int64_t *)ctx_buf(c, B_EOFF, sizeof(int64_t) * (size_t)(n + 2));
    int64_t *toff = (int64_t *)ctx_buf(c, B_K5_UNITS, sizeof(int64_t) * (size_t)(n + 2));
    if (!len || !toff || !task) return ESC_ENOMEM;
    k_wheel_tasks<<<grid_cap(c, n, 256), 256, 0, st>>>(n, (const int32_t *)c->buf[B_OFF], wq, c->wheel_split_deg, wk,
                                                       wd_lo, wflag, len);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, len, toff, n));
    int64_t nbig = 0;
    int32_t *town = nullptr;
    ESC_TRY(dev_task_owner(c, n, toff, &nbig, &town));
    auto kern = c->av ? k_wheels<true> : k_wheels<false>;
    ESC_TRY(run_sliced(c, "wheels", task + 8, task + 1, [&](uint64_t ticks) -> esc_status {
        kern<<<c->num_cu * per_cu, 64 * waves, lds, st>>>(
            n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int64_t *)c->buf[B_AOFF],
            (const uint32_t *)c->buf[B_AA], c->av, wq, wk, tab_words, toff, town, nbig, task + 4,
            c->task_chunk, c->wheel_split_deg, gmap_of(c), task + 1, tiny, (unsigned long long *)c->buf[B_ACC],
            (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 7, ticks, task + 8, wd_lo, wflag);
        HIP_TRY(hipGetLastError());
        return ESC_OK;
    }));
    ESC_TRY(mark_walk_end(c, STAGE_WHEELS));
    ESC_TRY(wheel_dense_product(c, dense));
    return ctx_release_if_short(c, {B_WD_Y});
}

esc_status stage_cycles(esc_ctx *c) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    if (n == 0 || c->m == 0) return ESC_OK;   // no 3-path: nothing to add, no tables to size
    uint32_t *tab;
    int32_t *touch;
    int *task;
    ESC_TRY(pair_scratch(c, &tab, &touch, &task));
    // the kernels with wave walks hold 94 (Y order) and 114 (Wnt order)
    // VGPRs, so two 8-wave workgroups per CU are resident: launch two, each
    // with the larger LDS slab; the one without (batches) keeps wg_per_cu
    const int per_cu = c->G ? c->wg_per_cu : slab_wgs_per_cu(c);
    int nwg = per_cu * c->num_cu;
    // two LDS arrays (X and Wnt) for the latest keys, leaving room for the static arrays
    const int32_t slab = slab_words(c, per_cu, 2, 8192, 13312);
    // a batch whose graphs are small takes a source per wave, with two
    // per-wave LDS tables over a graph's keys (16-bit counts at most)
    const int32_t pw_words = c->G && c->tab_n <= 4096 ? (c->tab_n + 1) / 2 : 0;
    const int32_t lds_words = 16 * pw_words > 2 * slab ? 16 * pw_words : (2 * slab > 0 ? 2 * slab : 1);
    // one graph with maximum degree below 2^16: the Y-table order (32-bit
    // Y(i,j) < d(i) d(j)), unless the Wnt order is asked for
    auto kern = c->G ? k_five_cycles<false, false>
                     : (c->maxdeg < 65536 && c->five_order == 0 ? k_five_cycles<true, true>
                                                                 : k_five_cycles<true, false>);
    return run_sliced(c, "five_cycles", task + 8, task + 2, [&](uint64_t ticks) -> esc_status {
        kern<<<nwg, 512, sizeof(uint32_t) * (size_t)lds_words, st>>>(
            n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_SPLIT], tab,
            tab + (size_t)c->tab_n * nwg, touch, touch + (size_t)c->tab_n * nwg, c->tab_n, c->task_chunk,
            gmap_of(c), task + 2, slab, pw_words, (unsigned long long *)c->buf[B_ACC],
            (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 8, ticks, task + 8);
        HIP_TRY(hipGetLastError());
        return ESC_OK;
    });
}
