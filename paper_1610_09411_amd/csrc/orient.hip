// Degree-ordered DAG (Sec. 2.2 of the paper): i precedes j when d(i) < d(j),
// ties broken by vertex id; every edge is oriented from the earlier to the
// later endpoint.  On the device the graph is relabelled by rank in that
// order, so "precedes" becomes "<" on the new ids, each sorted row holds the
// in-neighbours N-(v) as a prefix and the out-neighbours N+(v) as a suffix
// (split[v] marks the boundary), and every undirected edge gets the id of its
// out-arc.
//
// Kernels: validation + degrees, a stable LSD radix sort of vertices by degree,
// relabel + per-row sort (segmented bitonic sort), split points, edge ids and
// reverse arcs.  Also the generic device scan and segmented sort used by the
// later stages.
#include "device.h"
#include "ctx.h"

#define RS_THREADS 256
#define RS_ITEMS 16
#define RS_TILE (RS_THREADS * RS_ITEMS)

// ------------------------------------------------------------------ scan

template <typename T>
__global__ void __launch_bounds__(256) k_scan_block(const T *in, T *out, T *bsum, int64_t n_in, int64_t n_out) {
    __shared__ T part[256];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    T v[4];
    T s = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        int64_t idx = base + threadIdx.x * 4 + i;
        v[i] = (idx < n_in) ? in[idx] : (T)0;
        s += v[i];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        T y = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : (T)0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    T run = part[threadIdx.x] - s;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        int64_t idx = base + threadIdx.x * 4 + i;
        if (idx < n_out) out[idx] = run;
        run += v[i];
    }
    if (threadIdx.x == 255) bsum[blockIdx.x] = part[255];
}

template <typename T>
__global__ void k_scan_add(T *out, const T *bsum, int64_t n_out) {
    int64_t idx = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    T add = bsum[blockIdx.x];
    for (int i = 0; i < 4; i++, idx += 256)
        if (idx < n_out) out[idx] += add;
}

// exclusive scan of in[0..n) into out[0..n], out[n] = total.  `tmp` must hold
// enough for the block sums of every level (2 * (n/1024 + 64) elements).
template <typename T>
static esc_status scan_rec(hipStream_t st, const T *in, T *out, int64_t n_in, int64_t n_out, T *tmp) {
    int64_t nb = (n_out + 1023) / 1024;
    if (nb == 0) return ESC_OK;
    T *bsum = tmp;
    k_scan_block<T><<<dim3((unsigned)nb), dim3(256), 0, st>>>(in, out, bsum, n_in, n_out);
    HIP_TRY(hipGetLastError());
    if (nb > 1) {
        ESC_TRY(scan_rec<T>(st, bsum, bsum, nb, nb, tmp + nb + 64));
        k_scan_add<T><<<dim3((unsigned)nb), dim3(256), 0, st>>>(out, bsum, n_out);
        HIP_TRY(hipGetLastError());
    }
    return ESC_OK;
}

template <typename T>
static esc_status dev_scan(esc_ctx *c, const T *in, T *out, int64_t n) {
    T *tmp = (T *)ctx_buf(c, B_SCAN_TMP, sizeof(T) * (size_t)(2 * ((n + 1) / 1024 + 256)));
    if (!tmp) return ESC_ENOMEM;
    return scan_rec<T>(c->stream, in, out, n, n + 1, tmp);
}

esc_status dev_exclusive_scan_i64(esc_ctx *c, const int64_t *in, int64_t *out, int64_t n) {
    return dev_scan<int64_t>(c, in, out, n);
}

__global__ void k_task_owner(int32_t n, const int64_t *toff, int32_t *owner) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        for (int64_t u = toff[v]; u < toff[v + 1]; u++) owner[u] = v;
}

esc_status dev_task_owner(esc_ctx *c, int32_t n, const int64_t *toff, int64_t *ntasks, int32_t **owner) {
    HIP_TRY(hipMemcpyAsync(ntasks, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *owner = (int32_t *)ctx_buf(c, B_TASK_OWNER, sizeof(int32_t) * (size_t)(*ntasks + 1));
    if (!*owner) return ESC_ENOMEM;
    if (*ntasks == 0) return ESC_OK;
    k_task_owner<<<grid_cap(c, n, 256), 256, 0, c->stream>>>(n, toff, *owner);
    HIP_TRY(hipGetLastError());
    return ESC_OK;
}

// ----------------------------------------------------- validation, degrees

__global__ void k_degrees(int32_t n, const int32_t *rp, const int32_t *col, int32_t *deg, int *err,
                          int *maxdeg, int check) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int32_t a = rp[v], b = rp[v + 1];
        if (b < a) { atomicMax(err, (int)ESC_ERANGE); deg[v] = 0; continue; }
        deg[v] = b - a;
        atomicMax(maxdeg, b - a);
        if (!check) continue;
        for (int32_t p = a; p < b; p++) {
            int32_t x = col[p];
            if (x < 0 || x >= n) { atomicMax(err, (int)ESC_ERANGE); break; }
            if (x == v || (p > a && col[p - 1] >= x)) { atomicMax(err, (int)ESC_ENOTSIMPLE); break; }
        }
    }
}

// every arc (v,x) must have its reverse (x,v); run only on range-valid input
__global__ void k_symmetric(int32_t n, const int32_t *rp, const int32_t *col, int *err) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        for (int32_t p = rp[v]; p < rp[v + 1]; p++) {
            int32_t x = col[p];
            int32_t q = lower_bound_i32(col, rp[x], rp[x + 1], v);
            if (q >= rp[x + 1] || col[q] != v) { atomicMax(err, (int)ESC_ENOTSIMPLE); break; }
        }
    }
}

// ------------------------------------------------------- stable radix sort

// splitmix64 finaliser, used only for the random-order test hook
__device__ inline uint32_t mix32(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return (uint32_t)((z ^ (z >> 31)) >> 33);
}

__global__ void k_init_keys(int32_t n, const int32_t *deg, uint32_t *keys, uint32_t *vals, int random_order) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        keys[v] = random_order ? mix32((uint64_t)v) : (uint32_t)deg[v];
        vals[v] = (uint32_t)v;
    }
}

// batched calls: second sort key = graph of the vertex (stable on the first)
__global__ void k_graph_keys(int32_t n, const uint32_t *vals, const int32_t *vgraph, uint32_t *keys) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        keys[i] = (uint32_t)vgraph[vals[i]];
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint32_t *keys, int32_t n, int shift, int32_t *hist,
                                                        int32_t ntiles) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; i++) {
        int64_t idx = base + i * RS_THREADS + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: chunks of 256 elements in order; within a chunk
// equal digits are ranked by lane (ballot match) and by wave.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                                           uint32_t *vout, int32_t n, int shift,
                                                           const int32_t *hist_scan, int32_t ntiles) {
    __shared__ int32_t run[256];
    __shared__ int32_t wc[RS_THREADS / ESC_WAVE][256];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    run[threadIdx.x] = hist_scan[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    for (int i = 0; i < RS_ITEMS; i++) {
        for (int w = 0; w < RS_THREADS / ESC_WAVE; w++) wc[w][threadIdx.x] = 0;
        __syncthreads();
        int64_t idx = base + i * RS_THREADS + threadIdx.x;
        bool valid = idx < n;
        uint32_t key = valid ? kin[idx] : 0, val = valid ? vin[idx] : 0;
        uint32_t d = (key >> shift) & 255;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            uint64_t bm = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bm : ~bm;
        }
        int r = __popcll(peers & lt);
        if (valid && r == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t off = run[d] + r;
            for (int w = 0; w < wid; w++) off += wc[w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w = 0; w < RS_THREADS / ESC_WAVE; w++) add += wc[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void k_rank(int32_t n, const uint32_t *perm, int32_t *rank) {
    for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) rank[perm[r]] = r;
}

__global__ void k_rowlen(int32_t n, const uint32_t *perm, const int32_t *deg, int64_t *len) {
    for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) len[r] = deg[perm[r]];
}

// one wave per relabelled row
__global__ void k_fill_rows(int32_t n, const uint32_t *perm, const int32_t *rank, const int32_t *rp,
                            const int32_t *col, const int64_t *off64, int32_t *off, int32_t *adj) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t r = wave; r < n; r += nwaves) {
        int32_t v = (int32_t)perm[r];
        int32_t a = rp[v], b = rp[v + 1];
        int32_t o = (int32_t)off64[r];
        if (lane == 0) off[r] = o;
        for (int32_t p = a + lane; p < b; p += 64) adj[o + (p - a)] = rank[col[p]];
        if (r == n - 1 && lane == 0) off[n] = (int32_t)off64[n];
    }
}

__global__ void k_split(int32_t n, const int32_t *off, const int32_t *adj, int32_t *split, int64_t *dplus,
                        int *maxdplus) {
    for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        int32_t s = lower_bound_i32(adj, off[r], off[r + 1], r);
        split[r] = s;
        dplus[r] = off[r + 1] - s;
        atomicMax(maxdplus, off[r + 1] - s);
    }
}

// Work terms known once the degree order is (Thm fivevertex): wedges W, and
// the directed 3-paths i <- a -> b -> j counted with the j that close a
// triangle, sum over arcs a -> b of (d+(a) - 1) d+(b), taken at b over its
// in-neighbours a.  One thread per vertex b.
__global__ void k_work_terms(int32_t n, const int32_t *off, const int32_t *adj, const int32_t *split,
                             unsigned long long *w_out, unsigned long long *dp_out) {
    uint64_t w = 0, dp = 0;
    for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x) {
        const uint64_t d = (uint64_t)(off[b + 1] - off[b]), dpb = (uint64_t)(off[b + 1] - split[b]);
        w += c2(d);
        if (dpb == 0) continue;
        uint64_t s = 0;
        for (int32_t p = off[b]; p < split[b]; p++) {
            const int32_t a = adj[p];
            s += (uint64_t)(off[a + 1] - split[a] - 1);
        }
        dp += s * dpb;
    }
    flush_count(w, w_out);
    flush_count(dp, dp_out);
}

// edge id = index of the out-arc in the concatenation of all out-lists
__global__ void k_edges(int32_t n, const int32_t *off, const int32_t *adj, const int32_t *split,
                        const int64_t *eoff, int32_t *arc_eid, int32_t *rev, int32_t *earc, int32_t *elo) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        int32_t s = split[u], end = off[u + 1];
        int32_t e0 = (int32_t)eoff[u];
        for (int32_t p = s; p < end; p++) {
            int32_t v = adj[p];
            int32_t e = e0 + (p - s);
            int32_t q = lower_bound_i32(adj, off[v], split[v], u);
            arc_eid[p] = e;
            arc_eid[q] = e;
            rev[p] = q;
            rev[q] = p;
            earc[e] = p;
            elo[e] = u;
        }
    }
}

// --------------------------------------------------------- segmented sort

#define SEG_SMALL 32
#define SEG_WAVE 1024   // segments up to this length are sorted by one wave

#define SEG_PER_THREAD 8   // segments each thread classifies per tile

// Work lists of the segment classes.  A workgroup classifies a tile of
// blockDim * SEG_PER_THREAD segments: slots inside the tile come from LDS
// counters (one LDS atomic per wave and class), and the tile reserves its
// range of each class list with one global atomic per class; a global
// atomic per wave had serialised on the four counters.
__global__ void __launch_bounds__(256) k_seg_classify(const int64_t *seg_off, int64_t nseg, int32_t *q,
                                                      int32_t *counts, int64_t qcap, int64_t lds_keys) {
    __shared__ int lcnt[4], lbase[4];
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    const int64_t tile = (int64_t)blockDim.x * SEG_PER_THREAD;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < nseg; t0 += (int64_t)gridDim.x * tile) {
        if (threadIdx.x < 4) lcnt[threadIdx.x] = 0;
        __syncthreads();
        int cls[SEG_PER_THREAD], slot[SEG_PER_THREAD];
#pragma unroll
        for (int u = 0; u < SEG_PER_THREAD; u++) {
            const int64_t s = t0 + (int64_t)u * blockDim.x + threadIdx.x;
            cls[u] = -1;
            slot[u] = 0;
            if (s < nseg) {
                const int64_t len = seg_off[s + 1] - seg_off[s];
                if (len > 1) cls[u] = len <= SEG_SMALL ? 0 : (len <= SEG_WAVE ? 1 : (len <= lds_keys ? 2 : 3));
            }
            for (int c = 0; c < 4; c++) {
                const uint64_t m = __ballot(cls[u] == c);
                if (!m) continue;
                const int leader = __ffsll((long long)m) - 1;
                int b = 0;
                if (lane == leader) b = atomicAdd(&lcnt[c], __popcll(m));
                b = __shfl(b, leader);
                if (cls[u] == c) slot[u] = b + __popcll(m & lt);
            }
        }
        __syncthreads();
        if (threadIdx.x < 4) lbase[threadIdx.x] = lcnt[threadIdx.x] ? atomicAdd(&counts[threadIdx.x], lcnt[threadIdx.x]) : 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SEG_PER_THREAD; u++)
            if (cls[u] >= 0)
                q[cls[u] * qcap + lbase[cls[u]] + slot[u]] = (int32_t)(t0 + (int64_t)u * blockDim.x + threadIdx.x);
        __syncthreads();   // lcnt and lbase are reset by the next tile
    }
}

__global__ void k_seg_small(uint32_t *keys, const int64_t *seg_off, const int32_t *q, const int32_t *counts) {
    int32_t cnt = counts[0];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        int64_t s = q[i];
        int64_t a = seg_off[s];
        int len = (int)(seg_off[s + 1] - a);
        uint32_t v[SEG_SMALL];
        for (int j = 0; j < len; j++) v[j] = keys[a + j];
        for (int j = 1; j < len; j++) {
            uint32_t x = v[j];
            int k = j - 1;
            while (k >= 0 && v[k] > x) { v[k + 1] = v[k]; k--; }
            v[k + 1] = x;
        }
        for (int j = 0; j < len; j++) keys[a + j] = v[j];
    }
}

// medium segments: one wave sorts one segment (bitonic in its LDS region,
// wave-level barriers only)
__global__ void __launch_bounds__(256) k_seg_wave(uint32_t *keys, const int64_t *seg_off, const int32_t *q,
                                                  const int32_t *counts, int64_t qcap) {
    __shared__ uint32_t sk_all[4][SEG_WAVE];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t *sk = sk_all[wid];
    const int32_t cnt = counts[1];
    for (int32_t i = blockIdx.x * 4 + wid; i < cnt; i += gridDim.x * 4) {
        const int64_t s = q[qcap + i];
        const int64_t a = seg_off[s];
        const int len = (int)(seg_off[s + 1] - a);
        int N = 64;
        while (N < len) N <<= 1;
        for (int j = lane; j < N; j += 64) sk[j] = j < len ? keys[a + j] : 0xFFFFFFFFu;
        wave_sync();
        for (int k = 2; k <= N; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < N; t += 64) {
                    const int x = t ^ j;
                    if (x > t) {
                        const uint32_t p = sk[t], r = sk[x];
                        const bool asc = (t & k) == 0;
                        if ((p > r) == asc) { sk[t] = r; sk[x] = p; }
                    }
                }
                wave_sync();
            }
        for (int j = lane; j < len; j += 64) keys[a + j] = sk[j];
        wave_sync();
    }
}

// long segments: one workgroup per segment.  Keys that are distinct and
// span fewer than 32 x (the LDS words) values -- a triangle list holds
// distinct positions inside one row -- are sorted through a bitmap over
// [min, max]: set a bit per key, then every thread emits the set bits of
// its run of words at its place in the prefix count (O(len + span / 32),
// a few barriers).  Other segments (repeated keys: the popcount falls
// short of the length; a wider span) take the bitonic network in LDS.
__global__ void __launch_bounds__(256) k_seg_lds(uint32_t *keys, const int64_t *seg_off, const int32_t *q,
                                                 const int32_t *counts, int64_t qcap, int32_t lds_words) {
    extern __shared__ uint32_t sk[];
    __shared__ uint32_t rmin[4], rmax[4];
    __shared__ int tmp[8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t cnt = counts[2];
    for (int32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        int64_t s = q[2 * qcap + i];
        int64_t a = seg_off[s];
        int len = (int)(seg_off[s + 1] - a);
        // span of the keys
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        for (int j = threadIdx.x; j < len; j += blockDim.x) {
            const uint32_t k = keys[a + j];
            lo = k < lo ? k : lo;
            hi = k > hi ? k : hi;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
            lo = l2 < lo ? l2 : lo;
            hi = h2 > hi ? h2 : hi;
        }
        if (lane == 0) { rmin[wid] = lo; rmax[wid] = hi; }
        __syncthreads();
        lo = rmin[0];
        hi = rmax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) {
            lo = rmin[w] < lo ? rmin[w] : lo;
            hi = rmax[w] > hi ? rmax[w] : hi;
        }
        const uint64_t span = (uint64_t)hi - lo + 1;
        bool sorted = false;
        if (span <= 32ull * (uint64_t)lds_words) {
            const int nw = (int)((span + 31) >> 5);
            for (int w = threadIdx.x; w < nw; w += blockDim.x) sk[w] = 0;
            __syncthreads();
            for (int j = threadIdx.x; j < len; j += blockDim.x) {
                const uint32_t d = keys[a + j] - lo;
                atomicOr(&sk[d >> 5], 1u << (d & 31));
            }
            __syncthreads();
            // thread t owns words [t * per, (t + 1) * per)
            const int per = (nw + (int)blockDim.x - 1) / (int)blockDim.x;
            const int w0 = threadIdx.x * per, w1 = w0 + per < nw ? w0 + per : nw;
            int mine = 0;
            for (int w = w0; w < w1; w++) mine += __popc(sk[w]);
            int total;
            int pos = block_exclusive_scan(mine, tmp, &total);
            if (total == len) {   // distinct keys: the bitmap holds them all
                for (int w = w0; w < w1; w++) {
                    uint32_t x = sk[w];
                    while (x) {
                        const int b = __ffs(x) - 1;
                        x &= x - 1;
                        keys[a + pos++] = lo + (uint32_t)(w * 32 + b);
                    }
                }
                sorted = true;
            }
            __syncthreads();   // the bitmap is rewritten by the next segment or the network below
        }
        if (sorted) continue;
        int N = 1;
        while (N < len) N <<= 1;
        for (int j = threadIdx.x; j < N; j += blockDim.x) sk[j] = j < len ? keys[a + j] : 0xFFFFFFFFu;
        __syncthreads();
        for (int k = 2; k <= N; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = threadIdx.x; t < N; t += blockDim.x) {
                    int x = t ^ j;
                    if (x > t) {
                        uint32_t p = sk[t], r = sk[x];
                        bool asc = (t & k) == 0;
                        if ((p > r) == asc) { sk[t] = r; sk[x] = p; }
                    }
                }
                __syncthreads();
            }
        for (int j = threadIdx.x; j < len; j += blockDim.x) keys[a + j] = sk[j];
        __syncthreads();
    }
}

// rare very long segments: bitonic sort in a padded global buffer, one segment at a time
__global__ void __launch_bounds__(1024) k_seg_global(uint32_t *keys, const int64_t *seg_off, const int32_t *q,
                                                     const int32_t *counts, int64_t qcap, uint32_t *tmp) {
    int32_t cnt = counts[3];
    for (int32_t i = 0; i < cnt; i++) {
        int64_t s = q[3 * qcap + i];
        int64_t a = seg_off[s];
        int64_t len = seg_off[s + 1] - a;
        int64_t N = 1;
        while (N < len) N <<= 1;
        for (int64_t j = threadIdx.x; j < N; j += blockDim.x) tmp[j] = j < len ? keys[a + j] : 0xFFFFFFFFu;
        __syncthreads();
        for (int64_t k = 2; k <= N; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                for (int64_t t = threadIdx.x; t < N; t += blockDim.x) {
                    int64_t x = t ^ j;
                    if (x > t) {
                        uint32_t p = tmp[t], r = tmp[x];
                        bool asc = (t & k) == 0;
                        if ((p > r) == asc) { tmp[t] = r; tmp[x] = p; }
                    }
                }
                __syncthreads();
            }
        for (int64_t j = threadIdx.x; j < len; j += blockDim.x) keys[a + j] = tmp[j];
        __syncthreads();
    }
}

esc_status dev_segsort_u32(esc_ctx *c, uint32_t *keys, const int64_t *seg_off, int64_t nseg, int32_t maxlen) {
    if (nseg <= 0 || maxlen <= 1) return ESC_OK;
    int32_t *q = (int32_t *)ctx_buf(c, B_SEGQ, sizeof(int32_t) * (size_t)(4 * nseg + 16));
    int32_t *counts = (int32_t *)ctx_buf(c, B_SEGCLS, sizeof(int32_t) * 16);
    if (!q || !counts) return ESC_ENOMEM;
    hipStream_t st = c->stream;
    HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int32_t) * 16, st));
    int blocks = (int)((nseg + 255) / 256);
    if (blocks > 65535) blocks = 65535;
    // largest power-of-two key count one workgroup's LDS holds
    int64_t lds_keys = 1;
    while (lds_keys * 2 * (int64_t)sizeof(uint32_t) <= c->max_lds) lds_keys *= 2;
    const int64_t ctiles = (nseg + 256 * SEG_PER_THREAD - 1) / (256 * SEG_PER_THREAD);
    k_seg_classify<<<(int)(ctiles < 65535 ? (ctiles > 0 ? ctiles : 1) : 65535), 256, 0, st>>>(seg_off, nseg, q, counts,
                                                                                            nseg, lds_keys);
    HIP_TRY(hipGetLastError());
    k_seg_small<<<blocks, 256, 0, st>>>(keys, seg_off, q, counts);
    HIP_TRY(hipGetLastError());
    if (maxlen > SEG_SMALL) {
        k_seg_wave<<<c->num_cu * 8, 256, 0, st>>>(keys, seg_off, q, counts, nseg);
        HIP_TRY(hipGetLastError());
    }
    if (maxlen > SEG_WAVE) {
        int lds_n = 1;
        while (lds_n < maxlen && lds_n < lds_keys) lds_n <<= 1;
        int g = c->num_cu * 4;
        k_seg_lds<<<g, 256, sizeof(uint32_t) * lds_n, st>>>(keys, seg_off, q, counts, nseg, lds_n);
        HIP_TRY(hipGetLastError());
    }
    if (maxlen > lds_keys) {
        int64_t N = 1;
        while (N < maxlen) N <<= 1;
        uint32_t *tmp = (uint32_t *)ctx_buf(c, B_KEYS_B, sizeof(uint32_t) * (size_t)N);
        if (!tmp) return ESC_ENOMEM;
        k_seg_global<<<1, 1024, 0, st>>>(keys, seg_off, q, counts, nseg, tmp);
        HIP_TRY(hipGetLastError());
    }
    return ESC_OK;
}

// ------------------------------------------------------------ the stage

static int grid_for(esc_ctx *c, int64_t items, int threads) {
    int64_t b = (items + threads - 1) / threads;
    int64_t cap = (int64_t)c->num_cu * 16;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

esc_status stage_orient(esc_ctx *c, const int32_t *d_rp, const int32_t *d_col) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    c->key_w = c->key_dp = 0;
    int32_t *deg = (int32_t *)ctx_buf(c, B_DEG, sizeof(int32_t) * (size_t)(n + 1));
    int *err = (int *)ctx_buf(c, B_ERR, sizeof(int) * 4);
    if (!deg || !err) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(int) * 4, st));
    int check = (c->flags & ESC_F_VALIDATE) ? 1 : 0;
    k_degrees<<<grid_for(c, n, 256), 256, 0, st>>>(n, d_rp, d_col, deg, err, err + 1, check);
    HIP_TRY(hipGetLastError());
    int h_err[2];
    HIP_TRY(hipMemcpyAsync(h_err, err, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h_err[0]) return (esc_status)h_err[0];
    if (check) {
        k_symmetric<<<grid_for(c, n, 256), 256, 0, st>>>(n, d_rp, d_col, err);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h_err, err, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h_err[0]) return (esc_status)h_err[0];
    }
    c->maxdeg = h_err[1];

    // stable sort of vertices by (degree, id) -> perm; rank = inverse
    uint32_t *ka = (uint32_t *)ctx_buf(c, B_KEYS_A, sizeof(uint32_t) * (size_t)(n + 1));
    uint32_t *va = (uint32_t *)ctx_buf(c, B_VALS_A, sizeof(uint32_t) * (size_t)(n + 1));
    uint32_t *kb = (uint32_t *)ctx_buf(c, B_KEYS_B, sizeof(uint32_t) * (size_t)(n + 1));
    uint32_t *vb = (uint32_t *)ctx_buf(c, B_PERM, sizeof(uint32_t) * (size_t)(n + 1));
    int32_t ntiles = (int32_t)((n + RS_TILE - 1) / RS_TILE);
    int32_t *hist = (int32_t *)ctx_buf(c, B_HIST, sizeof(int32_t) * (size_t)(256 * (int64_t)ntiles + 1));
    int32_t *rank = (int32_t *)ctx_buf(c, B_RANK, sizeof(int32_t) * (size_t)(n + 1));
    if (!ka || !va || !kb || !vb || !hist || !rank) return ESC_ENOMEM;
    int random_order = (c->flags & ESC_F_RANDOM_ORDER) ? 1 : 0;
    k_init_keys<<<grid_for(c, n, 256), 256, 0, st>>>(n, deg, ka, va, random_order);
    HIP_TRY(hipGetLastError());
    int32_t *hs = (int32_t *)ctx_buf(c, B_TASK, sizeof(int32_t) * (size_t)(256 * (int64_t)ntiles + 2));
    if (!hs) return ESC_ENOMEM;
    // LSD radix sort, 8 bits per pass, ping-ponging between the two pairs:
    // first by degree (ties keep id order), then, for a batch, stably by graph
    uint32_t *kin = ka, *vin = va, *kout = kb, *vout = vb;
    for (int round = 0; round < (c->G ? 2 : 1) && n > 0; round++) {
        uint32_t maxkey = round ? (uint32_t)(c->G - 1) : random_order ? 0x7FFFFFFFu : (uint32_t)c->maxdeg;
        if (round) {
            k_graph_keys<<<grid_for(c, n, 256), 256, 0, st>>>(n, vin, (const int32_t *)c->buf[B_VGRAPH], kin);
            HIP_TRY(hipGetLastError());
        }
        int bits = 0;
        while (bits < 32 && (maxkey >> bits)) bits += 8;
        if (bits == 0) bits = 8;
        for (int pass = 0; pass < bits / 8; pass++) {
            int shift = pass * 8;
            k_rs_hist<<<ntiles, RS_THREADS, 0, st>>>(kin, n, shift, hist, ntiles);
            HIP_TRY(hipGetLastError());
            ESC_TRY(dev_scan<int32_t>(c, hist, hs, 256 * (int64_t)ntiles));
            k_rs_scatter<<<ntiles, RS_THREADS, 0, st>>>(kin, vin, kout, vout, n, shift, hs, ntiles);
            HIP_TRY(hipGetLastError());
            uint32_t *t;
            t = kin; kin = kout; kout = t;
            t = vin; vin = vout; vout = t;
        }
    }
    const uint32_t *perm = vin;   // B_VALS_A or B_PERM; the segmented sort below uses neither
    k_rank<<<grid_for(c, n, 256), 256, 0, st>>>(n, perm, rank);
    HIP_TRY(hipGetLastError());

    // relabelled CSR
    int64_t *len = (int64_t *)ctx_buf(c, B_EOFF, sizeof(int64_t) * (size_t)(n + 2));
    int64_t *off64 = (int64_t *)ctx_buf(c, B_AOFF, sizeof(int64_t) * (size_t)(n + 2));
    int32_t *off = (int32_t *)ctx_buf(c, B_OFF, sizeof(int32_t) * (size_t)(n + 1));
    int32_t *adj = (int32_t *)ctx_buf(c, B_ADJ, sizeof(int32_t) * (size_t)(c->m2 + 1));
    if (!len || !off64 || !off || !adj) return ESC_ENOMEM;
    k_rowlen<<<grid_for(c, n, 256), 256, 0, st>>>(n, perm, deg, len);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_scan<int64_t>(c, len, off64, n));
    if (n > 0) {
        k_fill_rows<<<grid_for(c, (int64_t)n * 64, 256), 256, 0, st>>>(n, perm, rank, d_rp, d_col, off64, off, adj);
        HIP_TRY(hipGetLastError());
        ESC_TRY(dev_segsort_u32(c, (uint32_t *)adj, off64, n, c->maxdeg));
    } else {
        HIP_TRY(hipMemsetAsync(off, 0, sizeof(int32_t), st));
    }

    // split points, edge ids, reverse arcs
    int32_t *split = (int32_t *)ctx_buf(c, B_SPLIT, sizeof(int32_t) * (size_t)(n + 1));
    int32_t *arc_eid = (int32_t *)ctx_buf(c, B_ARC_EID, sizeof(int32_t) * (size_t)(c->m2 + 1));
    int32_t *rev = (int32_t *)ctx_buf(c, B_REV, sizeof(int32_t) * (size_t)(c->m2 + 1));
    int32_t *earc = (int32_t *)ctx_buf(c, B_EARC, sizeof(int32_t) * (size_t)(c->m + 1));
    int32_t *elo = (int32_t *)ctx_buf(c, B_ELO, sizeof(int32_t) * (size_t)(c->m + 1));
    if (!split || !arc_eid || !rev || !earc || !elo) return ESC_ENOMEM;
    k_split<<<grid_for(c, n, 256), 256, 0, st>>>(n, off, adj, split, len, err + 2);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h_err, err + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    ESC_TRY(dev_scan<int64_t>(c, len, off64, n));   // off64 := out-arc offsets (edge ids)
    k_edges<<<grid_for(c, n, 256), 256, 0, st>>>(n, off, adj, split, off64, arc_eid, rev, earc, elo);
    HIP_TRY(hipGetLastError());
    unsigned long long *work = (unsigned long long *)c->buf[B_WORK];
    k_work_terms<<<grid_for(c, n, 256), 256, 0, st>>>(n, off, adj, split, work + WORK_W, work + WORK_DP);
    HIP_TRY(hipGetLastError());
    uint64_t terms[3] = {0, 0, 0};   // [WORK_DP], [WORK_DBP], [WORK_W]
    HIP_TRY(hipMemcpyAsync(terms, work + WORK_DP, sizeof(terms), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->maxdplus = h_err[0];
    c->key_dp = terms[0];
    c->key_w = terms[2];
    return ESC_OK;
}
