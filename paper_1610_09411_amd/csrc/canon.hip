// ESC_F_CANONICALIZE: turn any CSR (rows in any order, repeated entries,
// self-loops, arcs given in one direction only) into the simple undirected
// graph it describes, in sorted symmetric CSR, on the device.  Every entry
// (u,v) with u != v stands for the edge {u,v}; the result has each edge once
// in both rows, rows sorted.
#include <limits.h>
#include "device.h"
#include "ctx.h"

// one wave per input row: check ids, count both arcs of every non-loop entry
__global__ void k_can_count(int32_t n, const int32_t *rp, const int32_t *col, int32_t *cnt, int *err) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t u = wave; u < n; u += nwaves) {
        const int32_t a = rp[u], b = rp[u + 1];
        if (b < a) {
            if (lane == 0) atomicMax(err, (int)ESC_ERANGE);
            continue;
        }
        for (int32_t p = a + lane; p < b; p += 64) {
            const int32_t v = col[p];
            if (v < 0 || v >= n) { atomicMax(err, (int)ESC_ERANGE); continue; }
            if (v == u) continue;
            atomicAdd(&cnt[u], 1);
            atomicAdd(&cnt[v], 1);
        }
    }
}

__global__ void k_can_widen(int32_t n, const int32_t *cnt, int64_t *len, int *maxlen) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        len[u] = cnt[u];
        atomicMax(maxlen, cnt[u]);
    }
}

// scatter both arcs of every entry into their rows (unsorted within a row)
__global__ void k_can_fill(int32_t n, const int32_t *rp, const int32_t *col, const int64_t *off, int32_t *cur,
                           uint32_t *arcs) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t u = wave; u < n; u += nwaves) {
        const int32_t a = rp[u], b = rp[u + 1];
        for (int32_t p = a + lane; p < b; p += 64) {
            const int32_t v = col[p];
            if (v == u) continue;
            arcs[off[u] + atomicAdd(&cur[u], 1)] = (uint32_t)v;
            arcs[off[v] + atomicAdd(&cur[v], 1)] = (uint32_t)u;
        }
    }
}

// distinct entries of each sorted row: pass 0 counts them, pass 1 writes them
__global__ void k_can_unique(int32_t n, const int64_t *off, const uint32_t *arcs, int64_t *ulen,
                             const int64_t *uoff, int32_t *ocol, int pass) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int32_t u = wave; u < n; u += nwaves) {
        const int64_t a = off[u], b = off[u + 1];
        int64_t w = pass ? uoff[u] : 0;
        for (int64_t base = a; base < b; base += 64) {
            const int64_t p = base + lane;
            const bool keep = p < b && (p == a || arcs[p] != arcs[p - 1]);
            const uint64_t m = __ballot(keep);
            if (pass && keep) ocol[w + __popcll(m & lt)] = (int32_t)arcs[p];
            w += __popcll(m);
        }
        if (!pass && lane == 0) ulen[u] = w;
    }
}

__global__ void k_can_rows(int32_t n, const int64_t *uoff, int32_t *orp) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += gridDim.x * blockDim.x)
        orp[u] = (int32_t)uoff[u];
}

// d_rp / d_col: the input on the device.  On success *rp_out / *col_out
// point at the canonical CSR (context buffers) and *m2_out is its arc count.
esc_status canonicalize(esc_ctx *c, int32_t n, const int32_t *d_rp, const int32_t *d_col, const int32_t **rp_out,
                        const int32_t **col_out, int64_t *m2_out) {
    hipStream_t st = c->stream;
    int32_t *cnt = (int32_t *)ctx_buf(c, B_CAN_CNT, sizeof(int32_t) * ((size_t)n + 1));
    int64_t *len = (int64_t *)ctx_buf(c, B_CAN_LEN, sizeof(int64_t) * ((size_t)n + 2));
    int64_t *aoff = (int64_t *)ctx_buf(c, B_CAN_OFF, sizeof(int64_t) * ((size_t)n + 2));
    int64_t *uoff = (int64_t *)ctx_buf(c, B_CAN_UOFF, sizeof(int64_t) * ((size_t)n + 2));
    int *err = (int *)ctx_buf(c, B_ERR, sizeof(int) * 4);
    int32_t *orp = (int32_t *)ctx_buf(c, B_CAN_RP, sizeof(int32_t) * ((size_t)n + 1));
    if (!cnt || !len || !aoff || !uoff || !err || !orp) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ((size_t)n + 1), st));
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(int) * 4, st));
    const int gw = grid_cap(c, (int64_t)n * 64, 256), gt = grid_cap(c, n + 1, 256);
    // 1. arcs per row (both directions of every non-loop entry), their offsets
    if (n > 0) {
        k_can_count<<<gw, 256, 0, st>>>(n, d_rp, d_col, cnt, err);
        HIP_TRY(hipGetLastError());
        k_can_widen<<<gt, 256, 0, st>>>(n, cnt, len, err + 1);
        HIP_TRY(hipGetLastError());
    }
    int h_err[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h_err, err, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h_err[0]) return (esc_status)h_err[0];
    ESC_TRY(dev_exclusive_scan_i64(c, len, aoff, n));
    int64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, aoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    uint32_t *arcs = (uint32_t *)ctx_buf(c, B_CAN_ARCS, sizeof(uint32_t) * ((size_t)total + 1));
    if (!arcs) return ESC_ENOMEM;
    // 2. scatter, sort every row, count its distinct entries
    if (n > 0) {
        HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ((size_t)n + 1), st));
        k_can_fill<<<gw, 256, 0, st>>>(n, d_rp, d_col, aoff, cnt, arcs);
        HIP_TRY(hipGetLastError());
        ESC_TRY(dev_segsort_u32(c, arcs, aoff, n, h_err[1]));
        k_can_unique<<<gw, 256, 0, st>>>(n, aoff, arcs, len, nullptr, nullptr, 0);
        HIP_TRY(hipGetLastError());
    }
    ESC_TRY(dev_exclusive_scan_i64(c, len, uoff, n));
    int64_t m2 = 0;
    HIP_TRY(hipMemcpyAsync(&m2, uoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (m2 >= INT32_MAX) return ESC_ERANGE;
    int32_t *ocol = (int32_t *)ctx_buf(c, B_CAN_COL, sizeof(int32_t) * ((size_t)m2 + 1));
    if (!ocol) return ESC_ENOMEM;
    // 3. write the distinct entries and the row offsets
    if (n > 0) {
        k_can_unique<<<gw, 256, 0, st>>>(n, aoff, arcs, nullptr, uoff, ocol, 1);
        HIP_TRY(hipGetLastError());
    }
    k_can_rows<<<gt, 256, 0, st>>>(n, uoff, orp);
    HIP_TRY(hipGetLastError());
    *rp_out = orp;
    *col_out = ocol;
    *m2_out = m2;
    return ESC_OK;
}
