// Device-side helpers shared by the gfx950 kernels: exact 128-bit
// accumulation, block reductions and scans, load-balanced expansion of
// variable-length segments across a workgroup.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define ESC_WAVE 64

// Two 64-bit words hold one exact 128-bit sum.  Adding x: add the low word
// atomically; a wrap of that word is a carry into the high word.  Every
// individual addition detects its own wrap, so the total is exact.
__device__ inline void atomic_add_u128(unsigned long long *slot, u128 x) {
    unsigned long long lo = (unsigned long long)x;
    unsigned long long hi = (unsigned long long)(x >> 64);
    if (lo) {
        unsigned long long old = atomicAdd(slot, lo);
        if (old + lo < old) hi += 1;
    }
    if (hi) atomicAdd(slot + 1, hi);
}

__device__ inline u128 shfl_xor_u128(u128 x, int mask) {
    unsigned long long lo = (unsigned long long)x, hi = (unsigned long long)(x >> 64);
    lo = __shfl_xor(lo, mask);
    hi = __shfl_xor(hi, mask);
    return ((u128)hi << 64) | lo;
}

__device__ inline u128 wave_sum_u128(u128 x) {
    for (int o = ESC_WAVE / 2; o > 0; o >>= 1) x += shfl_xor_u128(x, o);
    return x;
}

// Sum NV 128-bit values over the block and add them to `slots[2*s]`.
// `scratch` must hold NV * (blockDim/64) u128 in LDS.
template <int NV>
__device__ inline void block_flush_u128(u128 (&v)[NV], u128 *scratch, unsigned long long *slots,
                                        const int *slot_ids) {
    const int lane = threadIdx.x & (ESC_WAVE - 1), wid = threadIdx.x / ESC_WAVE;
    const int nw = blockDim.x / ESC_WAVE;
#pragma unroll
    for (int s = 0; s < NV; s++) {
        u128 x = wave_sum_u128(v[s]);
        if (lane == 0) scratch[s * nw + wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        u128 t = 0;
        for (int w = 0; w < nw; w++) t += scratch[threadIdx.x * nw + w];
        if (t) atomic_add_u128(slots + 2 * slot_ids[threadIdx.x], t);
    }
    __syncthreads();
}

__device__ inline u128 shfl_up_u128(u128 x, int d) {
    unsigned long long lo = (unsigned long long)x, hi = (unsigned long long)(x >> 64);
    lo = __shfl_up(lo, d);
    hi = __shfl_up(hi, d);
    return ((u128)hi << 64) | lo;
}

// Batched calls keep one set of sums per graph (graph g at slots + g*stride).
// Each lane adds its NV values to the sums of its graph g; runs of adjacent
// lanes with the same g are summed first (segmented scan), so a wave whose
// lanes all hold one graph issues one atomic per value.  Lanes with g < 0
// hold nothing.  Zeroes v.  All 64 lanes of the wave must take part.
template <int NV>
__device__ inline void wave_flush_runs(u128 (&v)[NV], int g, unsigned long long *slots, size_t stride,
                                       const int *slot_ids) {
    const int lane = threadIdx.x & (ESC_WAVE - 1);
    const int gp = __shfl_up(g, 1);
    const uint64_t heads = __ballot(lane == 0 || gp != g);
    const uint64_t upto = heads & ((2ull << lane) - 1);       // run heads at or below this lane
    const int run0 = 63 - __clzll((long long)upto);
    const bool last = lane == ESC_WAVE - 1 || ((heads >> (lane + 1)) & 1);
#pragma unroll
    for (int s = 0; s < NV; s++) {
        u128 x = v[s];
        for (int o = 1; o < ESC_WAVE; o <<= 1) {
            u128 y = shfl_up_u128(x, o);
            if (lane - o >= run0) x += y;
        }
        if (last && g >= 0 && x) atomic_add_u128(slots + (size_t)g * stride + 2 * slot_ids[s], x);
        v[s] = 0;
    }
}

// Per-source kernels take whole sources per workgroup, so the graph of the
// current source is block-uniform: when it changes, the block's partial sums
// go to the graph they were gathered for.  Every thread of the block calls it.
template <int NV>
__device__ inline void block_switch_graph(u128 (&v)[NV], int &gcur, int gnew, u128 *scratch,
                                          unsigned long long *slots, size_t stride, const int *slot_ids) {
    if (gnew == gcur) return;
    if (gcur >= 0) {
        block_flush_u128<NV>(v, scratch, slots + (size_t)gcur * stride, slot_ids);
#pragma unroll
        for (int s = 0; s < NV; s++) v[s] = 0;
    }
    gcur = gnew;
}

// add the wave's sum of v to the 128-bit slot (one atomic, lane 0); zeroes v.
// Every lane of the wave must call it.
__device__ inline void wave_flush_u128(u128 &v, unsigned long long *slot) {
    const u128 x = wave_sum_u128(v);
    if ((threadIdx.x & (ESC_WAVE - 1)) == 0 && x) atomic_add_u128(slot, x);
    v = 0;
}

__device__ inline uint64_t wave_sum_u64(uint64_t x) {
    for (int o = ESC_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor((unsigned long long)x, o);
    return x;
}

// Exclusive scan of one int per thread over the block; returns the prefix and
// writes the total into *total.  `tmp` holds blockDim/64 + 1 ints in LDS.
__device__ inline int block_exclusive_scan(int x, int *tmp, int *total) {
    const int lane = threadIdx.x & (ESC_WAVE - 1), wid = threadIdx.x / ESC_WAVE;
    const int nw = blockDim.x / ESC_WAVE;
    int incl = x;
    for (int o = 1; o < ESC_WAVE; o <<= 1) {
        int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == ESC_WAVE - 1) tmp[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < nw; w++) { int t = tmp[w]; tmp[w] = run; run += t; }
        tmp[nw] = run;
    }
    __syncthreads();
    int res = tmp[wid] + incl - x;
    *total = tmp[nw];
    __syncthreads();
    return res;
}

// Spans of per-source work taken from a shared counter, sources in
// decreasing rank order.  The first TASK_HEAD grabs take `chunk` sources
// each (the high-rank sources, whose work varies most); every later grab
// takes TASK_TAIL, so the long tail of low-degree sources costs few atomics
// on the one counter.  Grab g covers [task_begin(g), task_begin(g + 1)).
#define TASK_HEAD 16384
#define TASK_TAIL 16
__device__ inline int64_t task_begin(int64_t g, int chunk) {
    return g < TASK_HEAD ? g * chunk : (int64_t)TASK_HEAD * chunk + (g - TASK_HEAD) * TASK_TAIL;
}

// Time slices of the per-source kernels.  A workgroup stops taking tasks
// once the wall clock passes slice_end (ticks of wall_clock64; 0 = no
// limit): the grab then returns GRAB_STOP, which maps past every task, so
// the workgroup finishes the tasks it holds and leaves; a later launch goes
// on from the shared counter.  A workgroup that sees the counter run out
// (a real grab past the end) sets *done: every task has then been taken by
// some workgroup of this launch, which completes it.
#define GRAB_STOP (1 << 30)
__device__ inline uint64_t slice_end_of(uint64_t slice_ticks) {
    return slice_ticks ? wall_clock64() + slice_ticks : 0;
}
__device__ inline int slice_grab(int *task, uint64_t slice_end) {
    if (slice_end && wall_clock64() > slice_end) return GRAB_STOP;
    return atomicAdd(task, 1);
}

// Load-balanced expansion.  A batch of up to blockDim segments, thread t
// describing segment t by (start, len); every element (segment s, position
// start_s + r) is visited exactly once, spread evenly over the block.
// `pref` and `beg` are LDS arrays of blockDim+1 entries, `tmp` as above
// with two more entries (blockDim / 64 + 2 in all).
//
// lbs_setup publishes the batch (prefixes, starts, total) and returns the
// total and the last non-empty segment (the one whose inclusive prefix
// reaches total: every later segment starts at total > x, so it bounds the
// searches; tmp[nw + 1] is free once the scan has returned).
__device__ inline int lbs_setup(int64_t start, int len, int *pref, int64_t *beg, int *tmp, int *last) {
    int total;
    int ex = block_exclusive_scan(len, tmp, &total);
    pref[threadIdx.x] = ex;
    beg[threadIdx.x] = start;
    if (threadIdx.x == 0) pref[blockDim.x] = total;
    if (len > 0 && ex + len == total) tmp[blockDim.x / ESC_WAVE + 1] = threadIdx.x;
    __syncthreads();
    *last = total > 0 ? tmp[blockDim.x / ESC_WAVE + 1] : 0;
    return total;
}

// element x's segment: the last one whose prefix is <= x.  A thread's x only
// grow, so the search goes on from its previous segment lo: one read while x
// stays in it (the segment's offset start - prefix stays in `base`), else a
// gallop and a halving past it.
__device__ inline void lbs_advance(const int *pref, const int64_t *beg, int last, int x, int &lo, int64_t &base) {
    if (lo < last && pref[lo + 1] <= x) {
        int a = lo + 1, step = 1;   // pref[a] <= x
        while (a + step <= last && pref[a + step] <= x) { a += step; step <<= 1; }
        int hi = a + step <= last ? a + step - 1 : last;
        while (a < hi) {
            const int mid = (a + hi + 1) >> 1;
            if (pref[mid] <= x) a = mid; else hi = mid - 1;
        }
        lo = a;
        base = beg[lo] - pref[lo];
    }
}

template <class Item>
__device__ inline void lbs_batch(int64_t start, int len, int *pref, int64_t *beg, int *tmp, Item item) {
    int last;
    const int total = lbs_setup(start, len, pref, beg, tmp, &last);
    int lo = 0;
    int64_t base = beg[0] - pref[0];
    for (int x = threadIdx.x; x < total; x += blockDim.x) {
        lbs_advance(pref, beg, last, x, lo, base);
        item(lo, base + x);
    }
    __syncthreads();
}

// add a per-thread count to a global counter, one atomic per wave
__device__ inline void flush_count(uint64_t x, unsigned long long *dst) {
    x = wave_sum_u64(x);
    if ((threadIdx.x & (ESC_WAVE - 1)) == 0 && x) atomicAdd(dst, (unsigned long long)x);
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lbs_batch with the element's read split from its use: load(q) reads the
// element at position q, use(s, q, v) consumes it.  A thread takes U of its
// elements at a time and issues their reads before any use, so U reads are
// in flight where an atomic use would otherwise wait for each read in turn.
template <int U, class L, class Use>
__device__ inline void lbs_batch_lu(int64_t start, int len, int *pref, int64_t *beg, int *tmp, L load, Use use) {
    int last;
    const int total = lbs_setup(start, len, pref, beg, tmp, &last);
    int lo = 0;
    int64_t base = beg[0] - pref[0];
    const int stride = (int)blockDim.x;
    for (int x0 = threadIdx.x; x0 < total; x0 += U * stride) {
        int ss[U];
        int64_t qq[U];
        decltype(load((int64_t)0)) vv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int x = x0 + u * stride;
            if (x < total) lbs_advance(pref, beg, last, x, lo, base);
            ss[u] = lo;
            qq[u] = base + x;
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            if (x0 + u * stride < total) vv[u] = load(qq[u]);
#pragma unroll
        for (int u = 0; u < U; u++)
            if (x0 + u * stride < total) use(ss[u], qq[u], vv[u]);
    }
    __syncthreads();
}

// A lane's place in the concatenation of a wave's 64 segments (LDS arrays
// sa = first position, se = exclusive and si = inclusive element prefix):
// the segment y holding element e is the first with si[y] > e.  Its end and
// the offset mapping e to a position (sa[y] - se[y]) stay in registers and
// are reloaded only when e passes the end, so a lane that stays inside one
// segment reads no LDS.  Elements are asked for in increasing order, all
// below si[63].
struct SegCursor {
    int y;
    int32_t end;
    int64_t base;
    __device__ inline void init(const int64_t *sa, const int32_t *se, const int32_t *si) {
        y = 0;
        end = si[0];
        base = sa[0] - se[0];
    }
    __device__ inline int64_t pos(int32_t e, const int64_t *sa, const int32_t *se, const int32_t *si) {
        if (end <= e) {
            do {
                y++;
                end = si[y];
            } while (end <= e);
            base = sa[y] - se[y];
        }
        return base + e;
    }
};

// Walk the concatenation of up to 64 segments held one per lane (lane y
// holds segment y = [a0, a1)), 64 consecutive elements per step, so that one
// step spans as many short segments as it needs; eight steps are issued
// before their results are used.  load(pos) reads the element at position
// pos, use(y, pos, value) consumes it (y = the lane holding the segment).
// sa/se/si are 64-entry LDS arrays private to the calling wave (the
// segments of one call hold fewer than 2^31 elements in all).  Every lane
// of the wave must call it.
template <int NU = 8, class L, class U>
__device__ inline void wave_walk_seg(int64_t a0, int64_t a1, int64_t *sa, int32_t *se, int32_t *si, L load, U use) {
    const int lane = threadIdx.x & (ESC_WAVE - 1);
    const int32_t len = (int32_t)(a1 - a0);
    int32_t incl = len;
    for (int o = 1; o < ESC_WAVE; o <<= 1) {
        const int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int32_t total = __shfl(incl, ESC_WAVE - 1);
    sa[lane] = a0;
    se[lane] = incl - len;
    si[lane] = incl;
    wave_sync();
    SegCursor c;
    c.init(sa, se, si);
    int32_t e = lane;
    // NU steps in flight
    for (; e + (NU - 1) * ESC_WAVE < total; e += NU * ESC_WAVE) {
        int64_t q[NU];
        int yy[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) {
            q[u] = c.pos(e + u * ESC_WAVE, sa, se, si);
            yy[u] = c.y;
        }
        decltype(load(q[0])) v[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) v[u] = load(q[u]);
#pragma unroll
        for (int u = 0; u < NU; u++) use(yy[u], q[u], v[u]);
    }
    for (; e < total; e += ESC_WAVE) {
        const int64_t q = c.pos(e, sa, se, si);
        use(c.y, q, load(q));
    }
    wave_sync();   // the arrays are reused by the next call
}

// wave_walk_seg with the use split in two: act(v) for the NU elements of a
// step first, then post(v, r) with r = act(v).  With an act that is one
// atomic and no branch, the NU atomics of a step are in flight together
// instead of each waiting for the branch of the one before.
template <class L, class A, class P>
__device__ inline void wave_walk_act(int64_t a0, int64_t a1, int64_t *sa, int32_t *se, int32_t *si, L load, A act,
                                     P post) {
    const int lane = threadIdx.x & (ESC_WAVE - 1);
    const int32_t len = (int32_t)(a1 - a0);
    int32_t incl = len;
    for (int o = 1; o < ESC_WAVE; o <<= 1) {
        const int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int32_t total = __shfl(incl, ESC_WAVE - 1);
    sa[lane] = a0;
    se[lane] = incl - len;
    si[lane] = incl;
    wave_sync();
    // each element's segment is looked up in LDS (no SegCursor): fewer
    // registers, and the wheel walks gain nothing from it
    int y = 0;
    int32_t e = lane;
    constexpr int NU = 8;   // steps in flight
    for (; e + (NU - 1) * ESC_WAVE < total; e += NU * ESC_WAVE) {
        int64_t q[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) {
            while (si[y] <= e + u * ESC_WAVE) y++;
            q[u] = sa[y] + (e + u * ESC_WAVE - se[y]);
        }
        decltype(load(q[0])) v[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) v[u] = load(q[u]);
        decltype(act(v[0])) r[NU];
#pragma unroll
        for (int u = 0; u < NU; u++) r[u] = act(v[u]);
#pragma unroll
        for (int u = 0; u < NU; u++) post(v[u], r[u]);
    }
    for (; e < total; e += ESC_WAVE) {
        while (si[y] <= e) y++;
        const auto v = load(sa[y] + (e - se[y]));
        post(v, act(v));
    }
    wave_sync();   // the arrays are reused by the next call
}

// wave_walk_seg with use(value) only
template <int NU = 8, class L, class U>
__device__ inline void wave_walk(int64_t a0, int64_t a1, int64_t *sa, int32_t *se, int32_t *si, L load, U use) {
    wave_walk_seg<NU>(a0, a1, sa, se, si, load, [&](int, int64_t, decltype(load(a0)) v) { use(v); });
}

// Same walk as wave_walk, counting for every segment the elements x with
// pred(load(pos)) true; returns the count of the calling lane's segment.
// cnt is a 64-entry LDS array private to the wave.
template <class L, class P>
__device__ inline uint32_t wave_count(int64_t a0, int64_t a1, int64_t *sa, int32_t *se, int32_t *si, uint32_t *cnt,
                                      L load, P pred) {
    const int lane = threadIdx.x & (ESC_WAVE - 1);
    const int32_t len = (int32_t)(a1 - a0);
    int32_t incl = len;
    for (int o = 1; o < ESC_WAVE; o <<= 1) {
        const int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int32_t total = __shfl(incl, ESC_WAVE - 1);
    sa[lane] = a0;
    se[lane] = incl - len;
    si[lane] = incl;
    cnt[lane] = 0;
    wave_sync();
    SegCursor c;
    c.init(sa, se, si);
    int ycur = 0;
    uint32_t run = 0;
    int32_t e = lane;
    for (; e + 3 * ESC_WAVE < total; e += 4 * ESC_WAVE) {
        int yy[4];
        int64_t q[4];
        for (int u = 0; u < 4; u++) {
            q[u] = c.pos(e + u * ESC_WAVE, sa, se, si);
            yy[u] = c.y;
        }
        const auto v0 = load(q[0]), v1 = load(q[1]), v2 = load(q[2]), v3 = load(q[3]);
        const uint32_t b[4] = {(uint32_t)pred(v0), (uint32_t)pred(v1), (uint32_t)pred(v2), (uint32_t)pred(v3)};
        for (int u = 0; u < 4; u++) {
            if (yy[u] != ycur) {
                if (run) atomicAdd(&cnt[ycur], run);
                run = 0;
                ycur = yy[u];
            }
            run += b[u];
        }
    }
    for (; e < total; e += ESC_WAVE) {
        const int64_t q = c.pos(e, sa, se, si);
        if (c.y != ycur) {
            if (run) atomicAdd(&cnt[ycur], run);
            run = 0;
            ycur = c.y;
        }
        run += (uint32_t)pred(load(q));
    }
    if (run) atomicAdd(&cnt[ycur], run);
    wave_sync();
    const uint32_t r = cnt[lane];
    wave_sync();   // the arrays are reused by the next call
    return r;
}

// Apex id of triangle-list entry q: the stored id, or, when the lists keep
// arc positions only (graphs whose lists would not fit twice), the
// neighbour at that position (av == nullptr).
__device__ inline int32_t apex_at(const int32_t *av, const int32_t *adj, const uint32_t *aa, int64_t q) {
    return av ? av[q] : adj[aa[q]];
}

// The same with the layout fixed at compile time (IDS: apex ids are stored),
// for kernels instantiated per layout: no test of av per entry.
template <bool IDS>
__device__ inline int32_t apex_at(const int32_t *av, const int32_t *adj, const uint32_t *aa, int64_t q) {
    return IDS ? av[q] : adj[aa[q]];
}

// Counts bounded by d pack 32 / 2^shift to a 32-bit word: 2-bit fields for
// d < 4, 4-bit for d < 16, 8-bit for d < 256, 16-bit for d < 2^16.
// Returns shift = log2(fields per word).
__device__ inline int count_shift(int64_t d) {
    return d < 4 ? 4 : (d < 16 ? 3 : (d < 256 ? 2 : (d < 65536 ? 1 : 0)));
}

__device__ inline uint64_t c2(uint64_t x) { return x < 2 ? 0 : x * (x - 1) / 2; }
// C(x,3) and C(x,4) without a 128-bit division (which compiles to a
// bit-serial loop): the factors 3 and 2 (resp. 3, 4 and 2) are divided out of
// the consecutive numbers that hold them, then the quotients are multiplied.
// Exact whenever the result fits 128 bits.
__device__ inline u128 c3(uint64_t x) {
    if (x < 3) return 0;
    uint64_t a = x, b = x - 1, c = x - 2;
    if (a % 3 == 0) a /= 3; else if (b % 3 == 0) b /= 3; else c /= 3;
    if ((a & 1) == 0) a >>= 1; else b >>= 1;   // dividing by 3 keeps the parity
    return (u128)a * b * c;
}
// Sum of C(f,3) over the cb-bit fields f of a packed word.  Only fields
// >= 3 are visited: some bit above the lowest two set, or both of those.
__device__ inline u128 c3_fields(uint32_t x, int cb, uint32_t cmask) {
    if (cb == 32) return c3(x);
    const uint32_t low = cb == 2 ? 0x55555555u : cb == 4 ? 0x11111111u : cb == 8 ? 0x01010101u : 0x00010001u;
    uint32_t hi = 0;
    for (int b = 2; b < cb; b++) hi |= x >> b;
    uint32_t m = (hi | (x & (x >> 1))) & low;
    u128 s = 0;
    while (m) {
        const int b = __builtin_ctz(m);
        s += c3((x >> b) & cmask);
        m &= m - 1;
    }
    return s;
}
__device__ inline u128 c4(uint64_t x) {
    if (x < 4) return 0;
    uint64_t f[4] = {x, x - 1, x - 2, x - 3};
    const int t = (int)(x % 3);                 // f[t] is a multiple of 3
    f[t] /= 3;                                  // keeps the residue mod 4 (3 is odd, 3^-1 = 3 mod 4)
    const int e = (int)(x & 1);                 // f[e] and f[e+2] are the even ones
    if ((f[e] & 3) == 0) { f[e] >>= 2; f[e + 2] >>= 1; } else { f[e] >>= 1; f[e + 2] >>= 2; }
    return (u128)f[0] * f[1] * f[2] * f[3];
}

// first index in sorted a[lo, hi) with a[idx] >= key
__device__ inline int lower_bound_i32(const int32_t *a, int lo, int hi, int32_t key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
