// Fragment counts of Thm 4vertex-tri and the linear cut-formula sums.
//
//  * triangles from out-wedges of the DAG (Thm 4vertex-tri): t(e) per edge,
//    then per-arc sorted triangle lists.  The list of arc (u->v) holds, for
//    every common neighbour w of u and v, the index of arc (u,w) in u's row;
//    the lists of an arc and of its reverse enumerate the same apexes in the
//    same order, which lets every triangle find all three of its arcs.
//  * 4-cycles (Thm 4cycle) from wedges below their latest vertex; only the
//    sums the 5-vertex formulas need (sum C4(e) t(e), sum C4(v)(d(v)-2)) are
//    formed, both linear in the per-edge counts.
//  * vertex and edge reductions for Thms 4vertex-easy, 5cutvertex, 5cutedge.
#include "device.h"
#include "ctx.h"

// ---------------------------------------------------------------- triangles

// One wave per vertex u.  N+(u) goes into a hash set in the wave's LDS
// (key: rank, value: position of the arc in u's row); the lanes take 64
// out-arcs u->v at a time and the wave walks the 64 lists N+(v) together,
// probing every entry x: a hit is the triangle u<v<x, found once, from its
// first arc.  Vertices whose N+ does not fit a wave's table take a whole
// workgroup's (k_triangles' first phase); beyond that they fall back to one
// merge per lane.
// mode 0: count t(e) (atomics on the three edges)
// mode 1: write the six per-arc list entries through per-arc cursors
__device__ inline uint32_t hash_slot(uint32_t x, int bits) { return (x * 2654435761u) >> (32 - bits); }

// With rec (mode 0), every triangle found is also recorded as its three
// arcs (u->v, u->w, v->w); the lists are then filled from the records
// (k_fill_records) instead of a second intersection.  The records go to
// TRI_REGIONS regions of rec_cap entries, one counter each (a single counter
// for the whole chip serialises its atomics); a record past its region's end
// sets the overflow word and is dropped (the caller then runs mode 1).
struct TriRec {
    int32_t p, x, y;
};
#define TRI_REGIONS 256
#define TRI_CSTRIDE 16   // u64 words between region counters (own cache lines)

// the six list entries of triangle u<v<w from arcs p=(u,v) x=(u,w) y=(v,w),
// each at a slot taken from its arc's cursor
__device__ inline void tri_fill6(const int32_t *rev, unsigned long long *cur, uint32_t *aa, int32_t p, int32_t x,
                                 int32_t y) {
    const int32_t rp = rev[p], rx = rev[x], ry = rev[y];
    aa[atomicAdd(&cur[p], 1ull)] = (uint32_t)x;    // list(u->v): apex w -> (u,w)
    aa[atomicAdd(&cur[rp], 1ull)] = (uint32_t)y;   // list(v->u): apex w -> (v,w)
    aa[atomicAdd(&cur[x], 1ull)] = (uint32_t)p;    // list(u->w): apex v -> (u,v)
    aa[atomicAdd(&cur[rx], 1ull)] = (uint32_t)ry;  // list(w->u): apex v -> (w,v)
    aa[atomicAdd(&cur[y], 1ull)] = (uint32_t)rp;   // list(v->w): apex u -> (v,u)
    aa[atomicAdd(&cur[ry], 1ull)] = (uint32_t)rx;  // list(w->v): apex u -> (w,u)
}

__device__ inline void tri_record(TriRec *rec, unsigned long long *rec_n, int64_t rec_cap, int region, int32_t p,
                                  int32_t x, int32_t y) {
    const unsigned long long k = atomicAdd(&rec_n[region * TRI_CSTRIDE], 1ull);
    if ((int64_t)k < rec_cap) {
        TriRec *r = rec + (int64_t)region * rec_cap + (int64_t)k;
        r->p = p;
        r->x = x;
        r->y = y;
    } else {
        atomicMax(&rec_n[TRI_REGIONS * TRI_CSTRIDE], 1ull);
    }
}

__device__ inline unsigned long long shfl_u64(unsigned long long v, int src) {
    const int lo = __shfl((int)(uint32_t)v, src), hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One step of a wave's walk over the lists N+(v) of 64 out-arcs pb + y of u:
// the lane's entry q (arc (v,w)) hit N+(u) at arc xw = (u,w), or xw < 0.  A
// step's lanes holding the same list y are consecutive; the first hit among
// them makes the one atomic the group needs on the arc pb + y (its count in
// mode 0, the slots of the group's entries in the lists of that arc and of
// its reverse in mode 1) and shares the result, so a dense list does not
// send 64 atomics to one address.  Every active lane of the step calls it.
// The active lanes need not be a prefix, nor their lists in order (the
// walk's last steps): a group is a run of active lanes with one list, and a
// lane whose lower neighbour is inactive starts one.
__device__ inline void tri_step(int mode, int32_t pb, int yl, int64_t q, int32_t xw, const int32_t *rev,
                                const int32_t *arc_eid, uint32_t *te, uint32_t *wcn, unsigned long long *cur,
                                uint32_t *aa, TriRec *rec, unsigned long long *rec_n, int64_t rec_cap, int region) {
    const int lane = threadIdx.x & 63;
    const bool hit = xw >= 0;
    const uint64_t hm = __ballot(hit);
    if (hm == 0) return;
    const uint64_t act = __ballot(1);
    const bool below_act = lane > 0 && ((act >> (lane - 1)) & 1);
    const int yprev = __shfl_up(yl, 1);
    const uint64_t heads = __ballot(!below_act || yprev != yl);
    const uint64_t before = (1ull << lane) - 1, upto = before | (1ull << lane);
    const int h0 = 63 - __clzll(heads & upto);                 // first lane of the lane's list
    const uint64_t later = heads & ~upto;                       // first lanes of the lists after it
    const uint64_t grp = hm & (later ? (later & (0ull - later)) - 1 : ~0ull) & ~((1ull << h0) - 1);
    const int rank = __popcll(grp & before), cnt = __popcll(grp);
    const int lead = grp ? __ffsll((long long)grp) - 1 : lane;
    const int32_t p = pb + yl, y = (int32_t)q;
    if (mode == 0) {
        if (hit) {
            atomicAdd(&te[arc_eid[xw]], 1u);
            atomicAdd(&te[arc_eid[y]], 1u);
            if (rank == 0) atomicAdd(&wcn[yl], (uint32_t)cnt);
            if (rec) tri_record(rec, rec_n, rec_cap, region, p, xw, y);
        }
        return;
    }
    unsigned long long s0 = 0, s1 = 0;
    if (hit && rank == 0) {
        s0 = atomicAdd(&cur[p], (unsigned long long)cnt);
        s1 = atomicAdd(&cur[rev[p]], (unsigned long long)cnt);
    }
    s0 = shfl_u64(s0, lead);
    s1 = shfl_u64(s1, lead);
    if (hit) {
        const int32_t rp = rev[p], rx = rev[xw], ry = rev[y];
        aa[s0 + rank] = (uint32_t)xw;                     // list(u->v): apex w -> (u,w)
        aa[s1 + rank] = (uint32_t)y;                      // list(v->u): apex w -> (v,w)
        aa[atomicAdd(&cur[xw], 1ull)] = (uint32_t)p;      // list(u->w): apex v -> (u,v)
        aa[atomicAdd(&cur[rx], 1ull)] = (uint32_t)ry;     // list(w->u): apex v -> (w,v)
        aa[atomicAdd(&cur[y], 1ull)] = (uint32_t)rp;      // list(v->w): apex u -> (v,u)
        aa[atomicAdd(&cur[ry], 1ull)] = (uint32_t)rx;     // list(w->v): apex u -> (w,u)
    }
}

// Vertices with 2 d+(u) above a wave's table but at most 2^big_hbits (the
// list big, *nbig of them) come first: workgroups take them from the counter
// grab, and N+(u) goes into one hash set over the LDS of all four waves'
// tables, which the waves probe as they walk the lists N+(v) of the out-arcs
// (64 arcs a wave at a time, in turn).  A workgroup with no such vertex left
// goes on to the others, so those vertices' triangles (in a dense core, most
// of the graph's) are found while the rest of the grid works.  Larger N+
// merge.
__global__ void __launch_bounds__(256) k_triangles(int32_t n, const int32_t *off, const int32_t *adj,
                                                   const int32_t *split, const int32_t *arc_eid,
                                                   const int32_t *rev, uint32_t *te, int mode,
                                                   unsigned long long *cur, uint32_t *aa, int hbits, int big_hbits,
                                                   const int32_t *big, const unsigned long long *nbig,
                                                   unsigned long long *grab, TriRec *rec,
                                                   unsigned long long *rec_n, int64_t rec_cap,
                                                   unsigned long long *visits) {
    extern __shared__ uint32_t hdyn[];   // per wave: keys[H] then values[H]
    __shared__ int64_t wsa[4][64];
    __shared__ int32_t wse[4][64], wsi[4][64];
    __shared__ uint32_t wcn[4][64];
    __shared__ int64_t s_t;
    uint64_t nvis = 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int H = 1 << hbits;
    const int region = blockIdx.x % TRI_REGIONS;
    auto fill6 = [&](int32_t p, int32_t x, int32_t y) { tri_fill6(rev, cur, aa, p, x, y); };
    auto record = [&](int32_t p, int32_t x, int32_t y) { tri_record(rec, rec_n, rec_cap, region, p, x, y); };
    wcn[wid][lane] = 0;
    if (big_hbits > 0) {
        // keys [0, 2^big_hbits), values after them: within the 4 x 2 x H words
        const int HB = 1 << big_hbits;
        uint32_t *bk = hdyn, *bv = hdyn + HB;
        for (int q = threadIdx.x; q < HB; q += blockDim.x) bk[q] = 0;
        const int64_t nb = (int64_t)*nbig;
        for (;;) {
            __syncthreads();   // the set is clear; s_t is free
            if (threadIdx.x == 0) s_t = (int64_t)atomicAdd(grab, 1ull);
            __syncthreads();
            const int64_t t = s_t;
            if (t >= nb) break;
            const int32_t u = big[t];
            const int32_t su = split[u], eu = off[u + 1];
            const int32_t dp = eu - su;   // 2^hbits < 2 dp <= 2^big_hbits
            int lb = hbits;
            while ((1 << lb) < 2 * dp) lb++;
            const uint32_t lm = (1u << lb) - 1;
            for (int32_t p = su + threadIdx.x; p < eu; p += blockDim.x) {
                const uint32_t x = (uint32_t)adj[p];
                uint32_t h = hash_slot(x, lb);
                while (atomicCAS(&bk[h], 0u, x + 1) != 0u) h = (h + 1) & lm;
                bv[h] = (uint32_t)p;
            }
            __syncthreads();
            auto find = [&](uint32_t x) -> int32_t {
                uint32_t h = hash_slot(x, lb);
                for (;;) {
                    const uint32_t k = bk[h];
                    if (k == x + 1) return (int32_t)bv[h];
                    if (k == 0) return -1;
                    h = (h + 1) & lm;
                }
            };
            for (int32_t pb = su + wid * 64; pb < eu; pb += nw * 64) {
                const int32_t p = pb + lane;
                int64_t a0 = 0, a1 = 0;
                if (p < eu) {
                    const int32_t v = adj[p];
                    a0 = split[v];
                    a1 = off[v + 1];
                }
                nvis += (uint64_t)(a1 - a0);
                wave_walk_seg(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return (uint32_t)adj[q]; },
                              [&](int yl, int64_t q, uint32_t w) {
                                  // find: arc (u,w) in u's row, or -1
                                  tri_step(mode, pb, yl, q, find(w), rev, arc_eid, te, wcn[wid], cur, aa, rec,
                                           rec_n, rec_cap, region);
                              });
                if (mode == 0) {
                    const uint32_t c = wcn[wid][lane];
                    if (c) {
                        atomicAdd(&te[arc_eid[p]], c);
                        wcn[wid][lane] = 0;
                    }
                    wave_sync();
                }
            }
            __syncthreads();   // every wave is done with the set
            for (int q = threadIdx.x; q <= (int)lm; q += blockDim.x) bk[q] = 0;
        }
    }
    uint32_t *hk = hdyn + (size_t)wid * 2 * H, *hv = hk + H;
    for (int q = lane; q < H; q += 64) hk[q] = 0;
    wave_sync();
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t u = wave; u < n; u += nwaves) {
        const int32_t su = split[u], eu = off[u + 1];
        const int32_t dp = eu - su;
        if (dp < 2) continue;
        if (2 * dp > H) {
            if (big_hbits > 0 && 2 * dp <= (1 << big_hbits)) continue;   // done in the first phase
            // merge fallback: lanes take the out-arcs u->v
            for (int32_t p = su + lane; p < eu; p += 64) {
                const int32_t v = adj[p];
                int32_t x = p + 1, y = split[v];
                const int32_t ev = off[v + 1];
                uint32_t cnt = 0;
                while (x < eu && y < ev) {
                    int32_t a = adj[x], b = adj[y];
                    nvis += 2;
                    if (a < b) x++;
                    else if (a > b) y++;
                    else {
                        if (mode == 0) {
                            atomicAdd(&te[arc_eid[x]], 1u);
                            atomicAdd(&te[arc_eid[y]], 1u);
                            cnt++;
                            if (rec) record(p, x, y);
                        } else {
                            fill6(p, x, y);
                        }
                        x++;
                        y++;
                    }
                }
                if (mode == 0 && cnt) atomicAdd(&te[arc_eid[p]], cnt);
            }
            continue;
        }
        int lb = 1;
        while ((1 << lb) < 2 * dp) lb++;
        const uint32_t lm = (1u << lb) - 1;
        for (int32_t p = su + lane; p < eu; p += 64) {
            const uint32_t x = (uint32_t)adj[p];
            uint32_t h = hash_slot(x, lb);
            while (atomicCAS(&hk[h], 0u, x + 1) != 0u) h = (h + 1) & lm;
            hv[h] = (uint32_t)p;
        }
        wave_sync();
        auto find = [&](uint32_t x) -> int32_t {
            uint32_t h = hash_slot(x, lb);
            for (;;) {
                const uint32_t k = hk[h];
                if (k == x + 1) return (int32_t)hv[h];
                if (k == 0) return -1;
                h = (h + 1) & lm;
            }
        };
        for (int32_t pb = su; pb < eu; pb += 64) {
            const int32_t p = pb + lane;
            int64_t a0 = 0, a1 = 0;
            if (p < eu) {
                const int32_t v = adj[p];
                a0 = split[v];
                a1 = off[v + 1];
            }
            nvis += (uint64_t)(a1 - a0);
            wave_walk_seg(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return (uint32_t)adj[q]; },
                          [&](int yl, int64_t q, uint32_t w) {
                              // find: arc (u,w) in u's row, or -1
                              tri_step(mode, pb, yl, q, find(w), rev, arc_eid, te, wcn[wid], cur, aa, rec, rec_n,
                                       rec_cap, region);
                          });
            if (mode == 0) {
                const uint32_t c = wcn[wid][lane];
                if (c) {
                    atomicAdd(&te[arc_eid[p]], c);
                    wcn[wid][lane] = 0;
                }
                wave_sync();
            }
        }
        for (int q = lane; q <= (int)lm; q += 64) hk[q] = 0;
        wave_sync();
    }
    if (visits) flush_count(nvis, visits);
}

// the vertices whose N+ takes a workgroup's hash set in k_triangles
__global__ void k_tri_big_list(int32_t n, const int32_t *off, const int32_t *split, int hbits, int big_hbits,
                               int32_t *big, unsigned long long *nbig) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const int32_t dp = off[u + 1] - split[u];
        if (2 * dp > (1 << hbits) && 2 * dp <= (1 << big_hbits)) big[atomicAdd(nbig, 1ull)] = u;
    }
}

// the six list entries of every recorded triangle u<v<w: it takes a slot on
// each of its three edges (a per-edge cursor; an arc and its reverse share
// their edge's slot), the lists are sorted afterwards
__global__ void k_fill_records(int64_t rec_cap, const TriRec *rec, const unsigned long long *rec_n,
                               const int32_t *rev, const int32_t *arc_eid, const int64_t *aoff, uint32_t *ecur,
                               uint32_t *aa) {
    const int64_t slots = rec_cap * TRI_REGIONS;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < slots; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t region = k / rec_cap;
        if (k - region * rec_cap >= (int64_t)rec_n[region * TRI_CSTRIDE]) continue;   // past the region's records
        const TriRec r = rec[k];
        const uint32_t sp = atomicAdd(&ecur[arc_eid[r.p]], 1u);
        const uint32_t sx = atomicAdd(&ecur[arc_eid[r.x]], 1u);
        const uint32_t sy = atomicAdd(&ecur[arc_eid[r.y]], 1u);
        const int32_t rp = rev[r.p], rx = rev[r.x], ry = rev[r.y];
        aa[aoff[r.p] + sp] = (uint32_t)r.x;    // list(u->v): apex w -> (u,w)
        aa[aoff[rp] + sp] = (uint32_t)r.y;     // list(v->u): apex w -> (v,w)
        aa[aoff[r.x] + sx] = (uint32_t)r.p;    // list(u->w): apex v -> (u,v)
        aa[aoff[rx] + sx] = (uint32_t)ry;      // list(w->u): apex v -> (w,v)
        aa[aoff[r.y] + sy] = (uint32_t)rp;     // list(v->w): apex u -> (v,u)
        aa[aoff[ry] + sy] = (uint32_t)rx;      // list(w->v): apex u -> (w,u)
    }
}

// sum over vertices of C(d+(v), 2): a bound on the triangle count
__global__ void k_wpp(int32_t n, const int32_t *off, const int32_t *split, unsigned long long *out) {
    uint64_t s = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        s += c2((uint64_t)(off[v + 1] - split[v]));
    flush_count(s, out);
}

// per arc: list length (= t of its edge) for the offsets, and t itself as a
// u32 array indexed like adj, so later passes read it sequentially
__global__ void k_arc_len(int64_t m2, const int32_t *arc_eid, const uint32_t *te, int64_t *len, uint32_t *tarc) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m2; p += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t = te[arc_eid[p]];
        len[p] = t;
        tarc[p] = t;
    }
}

__global__ void k_copy_cursor(int64_t m2, const int64_t *aoff, unsigned long long *cur) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m2; p += (int64_t)gridDim.x * blockDim.x)
        cur[p] = (unsigned long long)aoff[p];
}

__global__ void k_apex_ids(int64_t total, const uint32_t *aa, const int32_t *adj, int32_t *av) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x)
        av[k] = adj[aa[k]];
}

esc_status stage_triangles(esc_ctx *c) {
    const int32_t n = c->n;
    const int64_t m2 = c->m2, m = c->m;
    hipStream_t st = c->stream;
    const int32_t *off = (const int32_t *)c->buf[B_OFF], *adj = (const int32_t *)c->buf[B_ADJ];
    const int32_t *split = (const int32_t *)c->buf[B_SPLIT], *arc_eid = (const int32_t *)c->buf[B_ARC_EID];
    const int32_t *rev = (const int32_t *)c->buf[B_REV];
    uint32_t *te = (uint32_t *)ctx_buf(c, B_TE, sizeof(uint32_t) * (size_t)(m + 1));
    int64_t *len = (int64_t *)ctx_buf(c, B_EOFF, sizeof(int64_t) * (size_t)(m2 + 2));
    int64_t *aoff = (int64_t *)ctx_buf(c, B_AOFF, sizeof(int64_t) * (size_t)(m2 + 2));
    unsigned long long *cur = (unsigned long long *)ctx_buf(c, B_ACUR, sizeof(uint64_t) * (size_t)(m2 + 1));
    uint32_t *tarc = (uint32_t *)ctx_buf(c, B_TARC, sizeof(uint32_t) * (size_t)(m2 + 1));
    if (!te || !len || !aoff || !cur || !tarc) return ESC_ENOMEM;
    c->av = nullptr;
    HIP_TRY(hipMemsetAsync(te, 0, sizeof(uint32_t) * (size_t)(m + 1), st));
    if (n == 0) { c->narcs_apex = 0; return ESC_OK; }
    int g = grid_cap(c, (int64_t)n * 64, 256);
    unsigned long long *work = (unsigned long long *)c->buf[B_WORK];
    // per-wave hash sets of twice the largest out-degree, at most 2048 slots
    int hbits = 1;
    while ((1 << hbits) < 2 * c->maxdplus && hbits < 11) hbits++;
    const size_t hlds = sizeof(uint32_t) * 2 * 4 * ((size_t)1 << hbits);
    // Triangle records (12 B each, room for the bound sum C(d+(v),2)) when
    // they take at most an eighth of the free device memory and the lists
    // are not kept compact; otherwise the fill pass intersects again.
    // region counters, overflow word, the two passes' grab counters of the
    // big vertices, their count, bound
    const size_t ncnt = TRI_REGIONS * TRI_CSTRIDE + TRI_CSTRIDE + 4;
    unsigned long long *rcnt = (unsigned long long *)ctx_buf(c, B_TRICNT, sizeof(uint64_t) * ncnt);
    if (!rcnt) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(rcnt, 0, sizeof(uint64_t) * ncnt, st));
    k_wpp<<<grid_cap(c, n, 256), 256, 0, st>>>(n, off, split, rcnt + ncnt - 1);
    HIP_TRY(hipGetLastError());
    uint64_t wpp = 0;
    HIP_TRY(hipMemcpyAsync(&wpp, rcnt + ncnt - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    TriRec *rec = nullptr;
    // each region holds its share of the bound twice over (workgroups take
    // vertices in turn, so the regions fill about evenly)
    const int64_t rcap = (int64_t)(2 * wpp / TRI_REGIONS + 64);
    if (wpp > 0 && !(c->flags & ESC_F_COMPACT_LISTS)) {
        size_t fr = 0;
        ESC_TRY(ctx_free_bytes(c, &fr));
        const size_t want = sizeof(TriRec) * (size_t)rcap * TRI_REGIONS;
        if (want <= (fr + ctx_held(c, B_TRIREC)) / 8) rec = (TriRec *)ctx_buf(c, B_TRIREC, want);
    }
    // vertices with 2 d+ above a wave's table take their workgroup's four
    // (one set of at most 4 H slots: 2^13 with H = 2^11), listed first;
    // larger ones merge
    int big_hbits = 0;
    int32_t *big = nullptr;
    unsigned long long *nbig = rcnt + ncnt - 2;
    if (2 * (int64_t)c->maxdplus > (1 << hbits)) {
        big_hbits = hbits + 1;
        while ((1 << big_hbits) < 2 * c->maxdplus && big_hbits < hbits + 2) big_hbits++;
        // fewer than m / 2^(hbits-1) + 1 vertices have 2 d+ > 2^hbits
        big = (int32_t *)ctx_buf(c, B_TRIBIG, sizeof(int32_t) * (size_t)(m / ((int64_t)1 << (hbits - 1)) + 1));
        if (!big) return ESC_ENOMEM;
        k_tri_big_list<<<grid_cap(c, n, 256), 256, 0, st>>>(n, off, split, hbits, big_hbits, big, nbig);
        HIP_TRY(hipGetLastError());
    }
    k_triangles<<<g, 256, hlds, st>>>(n, off, adj, split, arc_eid, rev, te, 0, nullptr, nullptr, hbits, big_hbits,
                                      big, nbig, rcnt + ncnt - 4, rec, rcnt, rec ? rcap : 0,
                                      work + WORK_VISITS + 1);
    HIP_TRY(hipGetLastError());
    k_arc_len<<<grid_cap(c, m2, 256), 256, 0, st>>>(m2, arc_eid, te, len, tarc);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, len, aoff, m2));
    int64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, aoff + m2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->narcs_apex = total;
    // The lists hold arc positions (aa); the apex ids (av) are a copy for
    // faster reads, kept only when device memory has room for both beside
    // what the later stages allocate (per-edge K4, 5-clique bitmaps bounded
    // by m (max d+ / 64 + 1) words, per-workgroup tables, 4 GiB margin).
    const size_t list_bytes = sizeof(uint32_t) * (size_t)(total + 1);
    size_t later = sizeof(uint64_t) * (size_t)(m + 1) + 16 * (size_t)c->tab_n * (size_t)pair_wgs(c) + ((size_t)4 << 30);
    if (c->k == 5) later += sizeof(uint64_t) * (size_t)m * (size_t)(c->maxdplus / 64 + 1);
    size_t fr = 0;
    ESC_TRY(ctx_free_bytes(c, &fr));
    size_t avail = fr + ctx_held(c, B_AA) + ctx_held(c, B_AV);   // the two list buffers may be reallocated
    if (c->budget) {
        const size_t room = c->budget > c->held ? c->budget - c->held + ctx_held(c, B_AA) + ctx_held(c, B_AV) : 0;
        if (room < avail) avail = room;
    }
    // a no-allocation call keeps the compact layout: its region is small
    const bool keep_av = avail >= 2 * list_bytes + later && !(c->flags & ESC_F_COMPACT_LISTS) && !c->arena;
    if (!keep_av) ctx_release(c, B_AV);
    uint32_t *aa = (uint32_t *)ctx_buf(c, B_AA, list_bytes);
    int32_t *av = keep_av ? (int32_t *)ctx_buf(c, B_AV, list_bytes) : nullptr;
    if (!aa || (keep_av && !av)) return ESC_ENOMEM;
    c->av = av;
    if (total == 0) return ESC_OK;
    uint64_t overflow = 1;
    if (rec) {
        HIP_TRY(hipMemcpyAsync(&overflow, rcnt + TRI_REGIONS * TRI_CSTRIDE, sizeof(uint64_t), hipMemcpyDeviceToHost,
                               st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (rec && overflow == 0) {
        uint32_t *ecur = (uint32_t *)cur;   // m per-edge cursors in the per-arc cursor buffer
        HIP_TRY(hipMemsetAsync(ecur, 0, sizeof(uint32_t) * (size_t)(m + 1), st));
        k_fill_records<<<grid_cap(c, rcap * TRI_REGIONS, 256), 256, 0, st>>>(rcap, rec, rcnt, rev, arc_eid, aoff,
                                                                            ecur, aa);
        HIP_TRY(hipGetLastError());
    } else {
        k_copy_cursor<<<grid_cap(c, m2, 256), 256, 0, st>>>(m2, aoff, cur);
        HIP_TRY(hipGetLastError());
        k_triangles<<<g, 256, hlds, st>>>(n, off, adj, split, arc_eid, rev, te, 1, cur, aa, hbits, big_hbits, big,
                                          nbig, rcnt + ncnt - 3, nullptr, nullptr, 0, nullptr);
        HIP_TRY(hipGetLastError());
    }
    ESC_TRY(dev_segsort_u32(c, aa, aoff, m2, c->maxdeg));
    if (av) {
        k_apex_ids<<<grid_cap(c, total, 256), 256, 0, st>>>(total, aa, adj, av);
        HIP_TRY(hipGetLastError());
    }
    return ESC_OK;
}

// ------------------------------------------------------------------ 4-cycles

// One workgroup per top vertex h (latest vertex of the 4-cycle), taken from a
// shared counter, latest vertices first.  For every o before h the table
// holds c(h,o) = number of middles k (k before h, adjacent to h and o).
// Pass 1 counts, pass 2 revisits the wedges and reads c, pass 3 walks the
// touched keys:
//   C(c,2)                                       4-cycles
//   (c-1) * [t(hk) + t(ko)]   per wedge          sum_e C4(e) t(e)
//   (c-1) * (2 d(k) - 4)      per wedge   } sum_e C4(e)(d(u)+d(v)-4)
//   (c-1) * c * (d(h) + d(o) - 4)  per key }
// With per_edge set, pass 2 also adds c-1 to C4 of edges hk and ko.
//
// A top vertex with more than range_deg neighbours is taken by one workgroup
// and counted by key range: range r holds the keys o in [gb + r*R,
// gb + (r+1)*R) (R = the LDS slab in keys at h's packing), and passes 1 and 2
// read from every row N(k) only the run of keys in the range, so all counts
// of a range are in LDS.  Ranges go in key order, and each in-neighbour's run
// starts where its previous one ended (a cursor per in-neighbour in the
// workgroup's touched-key array, which pass 2 reads as well); the end is
// found by galloping from the start, so an empty run costs one element read
// (two binary searches per range and in-neighbour cost more than the runs
// themselves).  Without room for the cursors each run is found by binary
// searches.  Smaller tops go one per workgroup: keys in the latest `slab`
// ranks of h's graph are counted in LDS, the rest in the workgroup's dense
// table (relative to the graph's first rank).
__global__ void k_four_tasks(int32_t n, const int32_t *off, int32_t slab, int32_t range_deg, int64_t *len) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        len[v] = off[v + 1] - off[v] > range_deg && slab > 0 ? 1 : 0;
}

__global__ void __launch_bounds__(512) k_four_cycles(int32_t n, const int32_t *off, const int32_t *adj,
                                                     const int32_t *split, const int32_t *rev,
                                                     const int32_t *arc_eid, const uint32_t *tarc,
                                                     uint32_t *tab_all, int32_t *touch_all, int32_t tab_n,
                                                     const int64_t *toff, const int32_t *town, int64_t nbig,
                                                     int *task_big,
                                                     int chunk, GMap gm, int *task, int32_t slab,
                                                     int32_t range_deg, int32_t pw_words, unsigned long long *acc,
                                                     unsigned long long *c4e, unsigned long long *visits,
                                                     uint64_t slice_ticks, int *done) {
    extern __shared__ uint32_t sl[];
    uint64_t nvis = 0;
    const uint64_t slice_end = slice_end_of(slice_ticks);
    __shared__ int pref[513], tmp[16];
    __shared__ int64_t beg[513];
    __shared__ int s_h, s_nt;
    __shared__ u128 red[3 * 8];
    __shared__ int64_t wsa[8][64];
    __shared__ int32_t wse[8][64], wsi[8][64];
    uint32_t *Ct = tab_all + (size_t)blockIdx.x * tab_n;
    int32_t *touch = touch_all + (size_t)blockIdx.x * tab_n;
    const int ids[3] = {AC_C4, AC_N12, AC_N7X2};
    u128 sums[3] = {0, 0, 0};
    int gcur = -1;

    // large tops: one per workgroup, latest tops first, key ranges in order
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t u = nbig - 1 - slice_grab(task_big, slice_end);
            s_h = u >= 0 ? town[u] : -1;
        }
        __syncthreads();
        const int32_t h = s_h;
        __syncthreads();   // s_h is read by every thread before it is taken again
        if (h < 0) break;
        const int g = gm.graph(h);
        block_switch_graph<3>(sums, gcur, g, red, acc, ACC_STRIDE, ids);
        const int32_t oh = off[h], sh = split[h];
        const int64_t dh = off[h + 1] - oh;
        const int shift = count_shift(dh);
        const int cb = 32 >> shift;
        const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
        const int64_t rk = (int64_t)slab << shift;
        const int32_t gb = gm.begin(g);
        const int32_t nr = (int32_t)(((int64_t)(h - gb) + rk - 1) / rk);
        // the cursors: start and length of each in-neighbour's last run
        const bool keep = 2 * (int64_t)(sh - oh) <= tab_n;
        for (int32_t r = 0; r < nr; r++) {
            const int32_t o0 = (int32_t)(gb + r * rk);
            const int32_t o1 = (int32_t)(o0 + rk < h ? o0 + rk : h);
            const int32_t nwd = ((o1 - o0) + (1 << shift) - 1) >> shift;
            __syncthreads();   // the previous range's pass 3 is done with the slab
            for (int q = threadIdx.x; q < nwd; q += blockDim.x) sl[q] = 0;
            __syncthreads();
            auto slot = [&](int32_t o, uint32_t &s) -> uint32_t * {
                const int32_t idx = o - o0;
                s = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
                return &sl[idx >> shift];
            };
            // the run of row k below h with keys in [o0, o1)
            auto run = [&](int32_t p, int64_t &start, int &len) {
                start = 0;
                len = 0;
                if (p >= sh) return;
                const int32_t k = adj[p];
                int32_t a;
                if (!keep) {
                    a = lower_bound_i32(adj, off[k], rev[p], o0);
                } else {
                    const int32_t i = 2 * (p - oh);
                    a = r == 0 ? off[k] : touch[i] + touch[i + 1];   // rows hold only keys of k's graph
                }
                // first key >= o1 in [a, rev[p]): gallop from a, then halve
                const int64_t lim = rev[p];
                int64_t b = a;
                if (a < lim && adj[a] < o1) {
                    int64_t lo = a, step = 1;   // adj[lo] < o1
                    while (lo + step < lim && adj[lo + step] < o1) { lo += step; step <<= 1; }
                    int64_t hi = lo + step < lim ? lo + step : lim;
                    lo++;
                    while (lo < hi) { const int64_t mid = (lo + hi) >> 1; if (adj[mid] < o1) lo = mid + 1; else hi = mid; }
                    b = lo;
                }
                start = a;
                len = (int)(b - a);
                if (keep) {
                    touch[2 * (p - oh)] = a;
                    touch[2 * (p - oh) + 1] = len;
                }
            };
            // pass 1: counts
            for (int32_t base = oh; base < sh; base += blockDim.x) {
                int64_t start;
                int len;
                run(base + threadIdx.x, start, len);
                nvis += (uint64_t)len;
                lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                                [&](int, int64_t, int32_t o) {
                                    uint32_t s;
                                    uint32_t *w = slot(o, s);
                                    atomicAdd(w, 1u << s);
                                });
            }
            __syncthreads();
            // pass 2: per-wedge terms
            for (int32_t base = oh; base < sh; base += blockDim.x) {
                int64_t start = 0;
                int len = 0;
                if (!keep) {
                    run(base + threadIdx.x, start, len);
                } else if (base + (int32_t)threadIdx.x < sh) {
                    start = touch[2 * (base + threadIdx.x - oh)];
                    len = touch[2 * (base + threadIdx.x - oh) + 1];
                }
                lbs_batch_lu<4>(start, len, pref, beg, tmp, [&](int64_t q) { return adj[q]; },
                                [&](int s, int64_t q, int32_t o) {
                    const int32_t pk = base + s;
                    uint32_t sb;
                    const uint32_t cc = (*slot(o, sb) >> sb) & cmask;
                    if (cc >= 2) {
                        const int32_t k = adj[pk];
                        sums[1] += (uint64_t)(cc - 1) * (tarc[pk] + tarc[q]);
                        sums[2] += (uint64_t)(cc - 1) * (uint64_t)(2 * (off[k + 1] - off[k]) - 4);
                        if (c4e) {
                            atomicAdd(&c4e[arc_eid[pk]], (unsigned long long)(cc - 1));
                            atomicAdd(&c4e[arc_eid[q]], (unsigned long long)(cc - 1));
                        }
                    }
                });
            }
            // pass 3: per-key terms
            for (int q = threadIdx.x; q < nwd; q += blockDim.x) {
                const uint32_t x = sl[q];
                if (x == 0) continue;
                for (int f = 0; f < (1 << shift); f++) {
                    const uint64_t cc = (x >> (f * cb)) & cmask;
                    if (cc < 2) continue;
                    const int32_t o = o0 + (q << shift) + f;
                    sums[0] += c2(cc);
                    sums[2] += (u128)(cc - 1) * cc * (uint64_t)(dh + (off[o + 1] - off[o]) - 4);
                }
            }
        }
        __syncthreads();   // the touched-key array is read until pass 2 of the last range ends
    }

    if (pw_words > 0) {
        // a batch of small graphs: one top per wave, its counts in the wave's
        // own LDS table over the keys of its graph (pw_words words), so no
        // workgroup barrier per top
        if (gcur >= 0) {
            block_flush_u128<3>(sums, red, acc + (size_t)gcur * ACC_STRIDE, ids);
            sums[0] = sums[1] = sums[2] = 0;
        }
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
        uint32_t *wt = sl + (size_t)wid * pw_words;
        int wgc = -1;   // graph of the wave's sums
        for (;;) {
            if (threadIdx.x == 0) s_h = slice_grab(task, slice_end);
            __syncthreads();
            const int gi = s_h;
            const int64_t t0 = (int64_t)gi * chunk * nwv;
            __syncthreads();   // s_h is read by every thread before it is taken again
            if (t0 >= n) {
                if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
                break;
            }
            const int64_t t1 = t0 + (int64_t)chunk * nwv < n ? t0 + (int64_t)chunk * nwv : n;
            for (int64_t t = t0 + wid; t < t1; t += nwv) {
                const int32_t h = n - 1 - (int32_t)t;
                const int32_t oh = off[h], sh = split[h];
                const int64_t dh = off[h + 1] - oh;
                if (dh > range_deg && slab > 0) continue;   // done by key range
                if (sh - oh < 2) continue;                        // c(h,o) >= 2 needs two middles
                const int g = gm.graph(h);
                if (g != wgc) {
                    if (wgc >= 0) wave_flush_runs<3>(sums, wgc, acc, ACC_STRIDE, ids);
                    wgc = g;
                }
                const int32_t gb = gm.begin(g);
                const int shift = count_shift(dh);
                const int cb = 32 >> shift;
                const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
                const int32_t nwd = ((h - gb) + (1 << shift) - 1) >> shift;   // words of keys [gb, h)
                for (int q = lane; q < nwd; q += 64) wt[q] = 0;
                wave_sync();
                // pass 1: counts
                for (int32_t pb = oh; pb < sh; pb += 64) {
                    const int32_t p = pb + lane;
                    int64_t a0 = 0, a1 = 0;
                    if (p < sh) { a0 = off[adj[p]]; a1 = rev[p]; }
                    nvis += (uint64_t)(a1 - a0);
                    wave_walk(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return adj[q]; },
                              [&](int32_t o) {
                                  const int32_t idx = o - gb;
                                  atomicAdd(&wt[idx >> shift], 1u << ((idx & ((1 << shift) - 1)) * cb));
                              });
                }
                wave_sync();
                // pass 2: per-wedge terms
                for (int32_t pb = oh; pb < sh; pb += 64) {
                    const int32_t p = pb + lane;
                    int64_t a0 = 0, a1 = 0;
                    if (p < sh) { a0 = off[adj[p]]; a1 = rev[p]; }
                    wave_walk_seg(a0, a1, wsa[wid], wse[wid], wsi[wid], [&](int64_t q) { return adj[q]; },
                                  [&](int y, int64_t q, int32_t o) {
                                      const int32_t idx = o - gb;
                                      const uint32_t cc = (wt[idx >> shift] >> ((idx & ((1 << shift) - 1)) * cb)) & cmask;
                                      if (cc < 2) return;
                                      const int32_t pk = pb + y;
                                      const int32_t k = adj[pk];
                                      sums[1] += (uint64_t)(cc - 1) * (tarc[pk] + tarc[q]);
                                      sums[2] += (uint64_t)(cc - 1) * (uint64_t)(2 * (off[k + 1] - off[k]) - 4);
                                      if (c4e) {
                                          atomicAdd(&c4e[arc_eid[pk]], (unsigned long long)(cc - 1));
                                          atomicAdd(&c4e[arc_eid[q]], (unsigned long long)(cc - 1));
                                      }
                                  });
                }
                // pass 3: per-key terms
                for (int q = lane; q < nwd; q += 64) {
                    const uint32_t x = wt[q];
                    if (x == 0) continue;
                    for (int f = 0; f < (1 << shift); f++) {
                        const uint64_t cc = (x >> (f * cb)) & cmask;
                        if (cc < 2) continue;
                        const int32_t o = gb + (q << shift) + f;
                        sums[0] += c2(cc);
                        sums[2] += (u128)(cc - 1) * cc * (uint64_t)(dh + (off[o + 1] - off[o]) - 4);
                    }
                }
                wave_sync();   // the table is cleared by the wave's next top
            }
        }
        if (wgc >= 0) wave_flush_runs<3>(sums, wgc, acc, ACC_STRIDE, ids);
        flush_count(nvis, visits);
        return;
    }

    // smaller tops: one per workgroup
    if (threadIdx.x == 0) s_nt = 0;
    for (;;) {
        if (threadIdx.x == 0) s_h = slice_grab(task, slice_end);
        __syncthreads();
        const int gi = s_h;
        const int64_t t0 = task_begin(gi, chunk), tn = task_begin((int64_t)gi + 1, chunk);
        // s_h is read by every thread before it is taken again: a chunk whose
        // tops are all skipped has no other barrier before the next take
        __syncthreads();
        if (t0 >= n) {
            if (gi != GRAB_STOP && threadIdx.x == 0) *done = 1;
            break;
        }
        const int32_t t1 = (int32_t)(tn < n ? tn : n);
        for (int32_t t = (int32_t)t0; t < t1; t++) {
            const int32_t h = n - 1 - t;
            const int g = gm.graph(h);
            block_switch_graph<3>(sums, gcur, g, red, acc, ACC_STRIDE, ids);
            const int32_t gb = gm.begin(g), ge = gm.end(g);
            const int32_t oh = off[h], sh = split[h];
            const int64_t dh = off[h + 1] - oh;
            if (dh > range_deg && slab > 0) continue;   // done by key range
            // c(h,o) <= d(h): a low-degree top vertex packs 16, 8, 4 or 2
            // counts per word (count_shift), in LDS (that many times more
            // latest ranks) and in the table
            const int shift = count_shift(dh);
            const int cb = 32 >> shift;
            const uint32_t cmask = cb == 32 ? 0xFFFFFFFFu : (1u << cb) - 1u;
            const int32_t hi0 = ge - (slab << shift) > gb ? ge - (slab << shift) : gb;   // first key held in LDS
            const int32_t nsl = h > hi0 ? h - hi0 : 0;                                  // LDS keys [hi0, h)
            const int32_t nslw = (nsl + (1 << shift) - 1) >> shift;
            for (int q = threadIdx.x; q < nslw; q += blockDim.x) sl[q] = 0;
            __syncthreads();
            auto inc = [&](int32_t o) -> uint32_t {
                const int32_t idx = o >= hi0 ? o - hi0 : o - gb;
                const uint32_t s = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
                const uint32_t old = o >= hi0 ? atomicAdd(&sl[idx >> shift], 1u << s) : atomicAdd(&Ct[idx >> shift], 1u << s);
                return (old >> s) & cmask;
            };
            auto get = [&](int32_t o) -> uint32_t {
                const int32_t idx = o >= hi0 ? o - hi0 : o - gb;
                const uint32_t s = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
                return ((o >= hi0 ? sl[idx >> shift] : Ct[idx >> shift]) >> s) & cmask;
            };
            // pass 1: wedges h - k - o, k in N-(h), o in the prefix of N(k) below h
            for (int32_t base = oh; base < sh; base += blockDim.x) {
                int32_t p = base + threadIdx.x;
                int start = 0, len = 0;
                if (p < sh) { int32_t k = adj[p]; start = off[k]; len = rev[p] - off[k]; }
                lbs_batch(start, len, pref, beg, tmp, [&](int, int q) {
                    const int32_t o = adj[q];
                    nvis++;
                    if (inc(o) == 0 && o < hi0) touch[atomicAdd(&s_nt, 1)] = o;
                });
            }
            __syncthreads();
            // pass 2: per-wedge terms
            for (int32_t base = oh; base < sh; base += blockDim.x) {
                int32_t p = base + threadIdx.x;
                int start = 0, len = 0;
                if (p < sh) { int32_t k = adj[p]; start = off[k]; len = rev[p] - off[k]; }
                lbs_batch(start, len, pref, beg, tmp, [&](int s, int q) {
                    const int32_t pk = base + s;
                    const int32_t o = adj[q];
                    const uint32_t cc = get(o);
                    if (cc >= 2) {
                        const int32_t k = adj[pk];
                        sums[1] += (uint64_t)(cc - 1) * (tarc[pk] + tarc[q]);
                        sums[2] += (uint64_t)(cc - 1) * (uint64_t)(2 * (off[k + 1] - off[k]) - 4);
                        if (c4e) {
                            atomicAdd(&c4e[arc_eid[pk]], (unsigned long long)(cc - 1));
                            atomicAdd(&c4e[arc_eid[q]], (unsigned long long)(cc - 1));
                        }
                    }
                });
            }
            // pass 3: per-key terms, tables back to zero
            const int nt = s_nt;
            for (int i = threadIdx.x; i < nt + nsl; i += blockDim.x) {
                int32_t o;
                uint64_t cc;
                if (i < nt) {
                    o = touch[i];
                    const int32_t idx = o - gb;
                    const uint32_t s = (uint32_t)((idx & ((1 << shift) - 1)) * cb);
                    // other counts of the word may be cleared concurrently
                    cc = (atomicAnd(&Ct[idx >> shift], ~(cmask << s)) >> s) & cmask;
                } else {
                    o = hi0 + (i - nt);
                    cc = get(o);
                }
                if (cc >= 2) {
                    sums[0] += c2(cc);
                    sums[2] += (u128)(cc - 1) * cc * (uint64_t)(dh + (off[o + 1] - off[o]) - 4);
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) s_nt = 0;   // next read of s_nt is behind a barrier
        }
    }
    if (gcur >= 0) block_flush_u128<3>(sums, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    flush_count(nvis, visits);
}

esc_status stage_four(esc_ctx *c, bool per_edge_c4) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    if (n == 0 || c->m == 0) return ESC_OK;   // no wedge: no 4-cycle, no tables to size
    int nwg = pair_wgs(c);
    size_t per = (size_t)c->tab_n * sizeof(uint32_t);
    uint32_t *tab = (uint32_t *)ctx_buf(c, B_WG_SCRATCH, per * 2 * nwg);
    int32_t *touch = (int32_t *)ctx_buf(c, B_WG_TOUCH, per * 2 * nwg);
    int *task = (int *)ctx_buf(c, B_TASK, sizeof(int) * 16);
    if (!tab || !touch || !task) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(task, 0, sizeof(int) * 16, st));
    unsigned long long *c4e = nullptr;
    if (per_edge_c4) {
        c4e = (unsigned long long *)ctx_buf(c, B_C4E, sizeof(uint64_t) * (size_t)(c->m + 1));
        if (!c4e) return ESC_ENOMEM;
        HIP_TRY(hipMemsetAsync(c4e, 0, sizeof(uint64_t) * (size_t)(c->m + 1), st));
    }
    // LDS slab for the latest keys of a graph, leaving room for the static arrays
    const int32_t slab = slab_words(c, slab_wgs_per_cu(c), 1, 16384, 16384);
    // a batch whose graphs are small counts its smaller tops a wave each, in
    // per-wave LDS tables over a graph's keys (16-bit counts at most)
    const int32_t pw_words = c->G && c->tab_n <= 4096 ? (c->tab_n + 1) / 2 : 0;
    const int32_t lds_words = 8 * pw_words > slab ? 8 * pw_words : (slab > 0 ? slab : 1);
    // key-range tasks of the tops with more than four_range_deg neighbours
    int64_t *len = (int64_t *)ctx_buf(c, B_EOFF, sizeof(int64_t) * (size_t)(n + 2));
    int64_t *toff = (int64_t *)ctx_buf(c, B_K5_UNITS, sizeof(int64_t) * (size_t)(n + 2));
    if (!len || !toff) return ESC_ENOMEM;
    k_four_tasks<<<grid_cap(c, n, 256), 256, 0, st>>>(n, (const int32_t *)c->buf[B_OFF], slab, c->four_range_deg,
                                                      len);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, len, toff, n));
    int64_t nbig = 0;
    int32_t *town = nullptr;
    ESC_TRY(dev_task_owner(c, n, toff, &nbig, &town));
    return run_sliced(c, "four_cycles", task + 8, task, [&](uint64_t ticks) -> esc_status {
        k_four_cycles<<<slab_wgs_per_cu(c) * c->num_cu, 512, sizeof(uint32_t) * (size_t)lds_words, st>>>(
            n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_SPLIT],
            (const int32_t *)c->buf[B_REV], (const int32_t *)c->buf[B_ARC_EID], (const uint32_t *)c->buf[B_TARC],
            tab, touch, c->tab_n, toff, town, nbig, task + 4, c->task_chunk, gmap_of(c), task, slab,
            c->four_range_deg, pw_words, (unsigned long long *)c->buf[B_ACC], c4e,
            (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 2, ticks, task + 8);
        HIP_TRY(hipGetLastError());
        return ESC_OK;
    });
}

// -------------------------------------------------------------- reductions

// Item ranges of the flat per-vertex / per-edge kernels.  A single graph
// strides the whole grid over the items; a batch gives every wave one
// contiguous block of items, so a wave meets few graph boundaries and keeps
// its per-graph sums in registers in between.
struct WaveRange {
    int64_t base, end, step;
};

__device__ inline WaveRange wave_range(int64_t items, bool blocked) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    WaveRange r;
    if (blocked) {
        const int64_t per = ((items + nwaves - 1) / nwaves + 63) & ~(int64_t)63;
        r.base = wave * per;
        r.end = r.base + per < items ? r.base + per : items;
        r.step = 64;
    } else {
        r.base = wave * 64;
        r.end = items;
        r.step = nwaves * 64;
    }
    return r;
}

// per vertex r (rank ids): t(v) = half the sum of t(e) over its edges,
// K4(v) = a third of the sum of K4(e) = a sixth of the sum of k4e.
#define VR_BIG 32    // rows walked by a whole wave in the vertex sums

__global__ void __launch_bounds__(256) k_vertex_reduce(int32_t n, const int32_t *off, const int32_t *adj,
                                                       const int32_t *split, const int32_t *arc_eid,
                                                       const uint32_t *te, const unsigned long long *k4e,
                                                       uint64_t *tv, GMap gm, unsigned long long *acc,
                                                       uint64_t *work) {
    __shared__ u128 red[10 * 4];
    const int ids[10] = {AC_W, AC_S3, AC_S4, AC_TT, AC_N3, AC_N4, AC_N9, AC_N15, AC_SW, AC_TD};
    u128 s[10] = {0};
    uint64_t wpp = 0, wpm = 0, nvis = 0;
    const int lane = threadIdx.x & 63;
    const bool batched = gm.vg != nullptr;
    const WaveRange wr = wave_range(n, batched);
    int gcur = -1;
    for (int64_t base = wr.base; base < wr.end; base += wr.step) {
        const int32_t r = (int32_t)(base + lane);
        const bool ok = base + lane < wr.end;
        if (batched) {
            const int g = ok ? gm.graph(r) : gcur;
            if (__ballot(g != gcur && gcur >= 0)) wave_flush_runs<10>(s, gcur, acc, ACC_STRIDE, ids);
            gcur = g;
        }
        const int32_t a = ok ? off[r] : 0, b = ok ? off[r + 1] : 0;
        const uint64_t d = b - a;
        uint64_t t2 = 0, k3 = 0, A = 0, sd = 0;
        u128 B = 0;
        auto arc_terms = [&](int32_t p, uint64_t &xt2, uint64_t &xk3, uint64_t &xA, u128 &xB, uint64_t &xsd) {
            const int32_t e = arc_eid[p];
            xt2 += te[e];
            xk3 += k4e[e];
            const int32_t j = adj[p];
            const uint64_t dj = off[j + 1] - off[j];
            xA += dj - 1;
            xB += (u128)(dj - 1) * (dj - 1);
            xsd += dj;
        };
        // a lane walks the row of its vertex; rows longer than VR_BIG are
        // walked by the whole wave (one lane alone would hold up the grid)
        const bool big = d > VR_BIG;
        if (ok && !big)
            for (int32_t p = a; p < b; p++) arc_terms(p, t2, k3, A, B, sd);
        for (uint64_t bm = __ballot(ok && big); bm; bm &= bm - 1) {
            const int L = __ffsll((long long)bm) - 1;
            const int32_t aL = __shfl(a, L), bL = __shfl(b, L);
            uint64_t pt2 = 0, pk3 = 0, pA = 0, psd = 0;
            u128 pB = 0;
            for (int32_t p = aL + lane; p < bL; p += 64) arc_terms(p, pt2, pk3, pA, pB, psd);
            pt2 = wave_sum_u64(pt2);
            pk3 = wave_sum_u64(pk3);
            pA = wave_sum_u64(pA);
            psd = wave_sum_u64(psd);
            pB = wave_sum_u128(pB);
            if (lane == L) { t2 = pt2; k3 = pk3; A = pA; B = pB; sd = psd; }
        }
        if (!ok) continue;
        nvis += d;
        const uint64_t t = t2 / 2, k4v = k3 / 6;
        tv[r] = t;
        s[0] += c2(d);
        s[1] += c3(d);
        s[2] += c4(d);
        if (t) s[3] += (u128)t * (d - 2);
        s[4] += ((u128)A * A - B) / 2;
        if (t && d >= 4) s[5] += (u128)t * c2(d - 2);
        s[6] += c2(t);
        if (d >= 3) s[7] += (u128)k4v * (d - 3);
        s[8] += (u128)c2(d) * d + (u128)(d ? d - 1 : 0) * sd;
        s[9] += (u128)t * d;
        const uint64_t dp = b - split[r], dm = split[r] - a;
        wpp += c2(dp);
        wpm += dp * dm;
    }
    if (batched) wave_flush_runs<10>(s, gcur, acc, ACC_STRIDE, ids);
    else block_flush_u128<10>(s, red, acc, ids);
    wpp = wave_sum_u64(wpp);
    wpm = wave_sum_u64(wpm);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long *)&work[0], (unsigned long long)wpp);
        atomicAdd((unsigned long long *)&work[1], (unsigned long long)wpm);
    }
    flush_count(nvis, (unsigned long long *)&work[WORK_VISITS + 5]);
}

__global__ void __launch_bounds__(256) k_edge_reduce(int64_t m, const int32_t *off, const int32_t *adj,
                                                     const int32_t *earc, const int32_t *elo, const uint32_t *te,
                                                     const uint64_t *tv, const unsigned long long *k4e, GMap gm,
                                                     unsigned long long *acc) {
    __shared__ u128 red[9 * 4];
    const int ids[9] = {AC_T3, AC_D, AC_EP, AC_N2, AC_N5, AC_N6, AC_N11, AC_N14, AC_N19};
    u128 s[9] = {0};
    const int lane = threadIdx.x & 63;
    const bool batched = gm.vg != nullptr;
    const WaveRange wr = wave_range(m, batched);
    int gcur = -1;
    for (int64_t base = wr.base; base < wr.end; base += wr.step) {
        const int64_t e = base + lane;
        const bool ok = e < wr.end;
        const int32_t u = ok ? elo[e] : 0;
        if (batched) {
            const int g = ok ? gm.graph(u) : gcur;
            if (__ballot(g != gcur && gcur >= 0)) wave_flush_runs<9>(s, gcur, acc, ACC_STRIDE, ids);
            gcur = g;
        }
        if (!ok) continue;
        const int32_t v = adj[earc[e]];
        const uint64_t du = off[u + 1] - off[u], dv = off[v + 1] - off[v];
        const uint64_t t = te[e], tu = tv[u], tw = tv[v], k4 = k4e[e] / 2;
        s[0] += t;
        s[1] += c2(t);
        s[2] += (u128)(du - 1) * (dv - 1);
        s[3] += (u128)(dv - 1) * c2(du - 1) + (u128)(du - 1) * c2(dv - 1);
        s[4] += (u128)(du - 1) * (tw - t) + (u128)(dv - 1) * (tu - t);
        if (t) s[5] += (u128)t * (du - 2) * (dv - 2);
        if (t >= 2) s[6] += (u128)c2(t) * ((du - 3) + (dv - 3));
        s[7] += c3(t);
        if (t >= 2) s[8] += (u128)k4 * (t - 2);
    }
    if (batched) wave_flush_runs<9>(s, gcur, acc, ACC_STRIDE, ids);
    else block_flush_u128<9>(s, red, acc, ids);
}

esc_status stage_reduce(esc_ctx *c) {
    hipStream_t st = c->stream;
    const int32_t n = c->n;
    const int64_t m = c->m;
    uint64_t *tv = (uint64_t *)ctx_buf(c, B_TV, sizeof(uint64_t) * (size_t)(n + 1));
    if (!tv) return ESC_ENOMEM;
    unsigned long long *acc = (unsigned long long *)c->buf[B_ACC];
    if (n > 0) {
        k_vertex_reduce<<<grid_cap(c, n, 256), 256, 0, st>>>(
            n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_SPLIT],
            (const int32_t *)c->buf[B_ARC_EID], (const uint32_t *)c->buf[B_TE],
            (const unsigned long long *)c->buf[B_K4E], tv, gmap_of(c), acc, (uint64_t *)c->buf[B_WORK]);
        HIP_TRY(hipGetLastError());
    }
    if (m > 0) {
        k_edge_reduce<<<grid_cap(c, m, 256), 256, 0, st>>>(
            m, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_EARC],
            (const int32_t *)c->buf[B_ELO], (const uint32_t *)c->buf[B_TE], tv,
            (const unsigned long long *)c->buf[B_K4E], gmap_of(c), acc);
        HIP_TRY(hipGetLastError());
    }
    return ESC_OK;
}
