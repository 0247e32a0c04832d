// Tiles of Y Y^T for 0/1 matrices on the matrix cores (gfx950): the
// products of pairs of hubs (pattern 17), of the neighbourhood of a hub with
// itself (wheels) and of the out-neighbourhood rows of a vertex over its
// neighbourhood (4-cliques per triangle).  Entries are 4-bit floats (e2m1:
// 0 and 1.0 = 0b0010), two to a byte, multiplied by the scaled f8f6f4
// instruction with unit scales into f32 accumulators: every product is 0 or
// 1 and every sum here stays below 2^24 (a row holds at most 2^17 entries),
// so the f32 results are exact integers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HUB_T 256      // tile of the product (rows and columns)
#define HUB_K 128      // bytes of a row staged per step (256 entries)
#ifndef HUB_WAVES
#define HUB_WAVES 8    // waves of a tile's workgroup (4 or 8)
#endif
#define HUB_WC (2 * HUB_T / HUB_WAVES)   // columns of a wave's part
#define HUB_BC (HUB_WC / 16)             // 16 x 16 products across a wave's part

typedef int hub_v4i __attribute__((ext_vector_type(4)));
typedef int hub_v8i __attribute__((ext_vector_type(8)));
typedef float hub_v4f __attribute__((ext_vector_type(4)));

// entry e of a row of 32-bit words set to 1.0 (e2m1 0b0010), 8 to a word
__device__ inline void fp4_set_one(uint32_t *row, int64_t e) { atomicOr(&row[e >> 3], 2u << ((e & 7) * 4)); }

// 16 x 16 x 128 product of 4-bit-float fragments (16 bytes a lane, the
// upper half of the operand registers unused), scales 2^0
__device__ inline hub_v4f hub_mfma(hub_v4i a, hub_v4i b, hub_v4f c) {
    const hub_v8i a8 = {a[0], a[1], a[2], a[3], 0, 0, 0, 0}, b8 = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
}

// Tiles of the hub-pair product are grouped in patches of HUB_PR x HUB_PC
// tiles (a patch of tile rows and columns with at least one tile on or above
// the diagonal); patch p goes to XCD p mod 8 (workgroup b runs on XCD b mod
// 8), its tiles to consecutive workgroups of that XCD, so the 32 CUs of an
// XCD hold one patch at a time and read each of its HUB_PR row blocks and
// HUB_PC column blocks once into their shared L2.
#define HUB_PR 4
#define HUB_PC 8

// number of patches with a tile on or above the diagonal, and patch p's
// first tile row and column
__host__ __device__ inline int hub_patch_rows(int nb) { return (nb + HUB_PR - 1) / HUB_PR; }
__host__ __device__ inline int hub_patch_cols(int nb) { return (nb + HUB_PC - 1) / HUB_PC; }
__host__ __device__ inline int hub_npatches(int nb) {
    int t = 0;
    for (int a = 0; a < hub_patch_rows(nb); a++) {
        const int c0 = (a * HUB_PR) / HUB_PC;   // first patch column reaching tile column a * HUB_PR
        t += hub_patch_cols(nb) - c0;
    }
    return t;
}

typedef __attribute__((address_space(3))) uint8_t lds_u8;

// One step of operand bytes into an LDS buffer by direct global -> LDS
// loads: the step's HUB_K bytes of the tile's 2 x HUB_T rows, as 64 loads
// of 8 rows (1 KB, 16 bytes a lane, the lanes' bytes land one after the
// other from the wave's LDS address), 64 / HUB_WAVES per wave.  Row r keeps its 16-byte
// chunk c at chunk position c ^ (r & 7) of its 128 LDS bytes, so the 8 rows
// a fragment read touches at one chunk fall in distinct banks.
__device__ inline void hub_stage(lds_u8 *buf, const uint8_t *ya, const uint8_t *yb, int32_t kb, int32_t k0, int wid,
                                 int lane) {
#pragma unroll
    for (int u8 = 0; u8 < 64 / HUB_WAVES; u8++) {
        const int u = wid * (64 / HUB_WAVES) + u8;       // load number, 0..63
        const int op = u >> 5, r0 = (u & 31) * 8;        // operand (A, B), first row
        const int row = r0 + (lane >> 3), cpos = lane & 7;
        const int cc = cpos ^ (row & 7);                 // the chunk that lands at cpos
        const uint8_t *g = (op ? yb : ya) + (size_t)row * kb + k0 + cc * 16;
        __builtin_amdgcn_global_load_lds((const void *)g, (lds_u8 *)(buf + op * HUB_T * HUB_K + r0 * HUB_K), 16, 0, 0);
    }
}

// fragment of 16 rows from `row0` of one operand in an LDS buffer: lane
// takes row row0 + (lane & 15), bytes kk + (lane >> 4) * 16 of the step
__device__ inline hub_v4i hub_frag(const lds_u8 *opb, int row0, int kk, int lane) {
    const int row = row0 + (lane & 15), c = (kk >> 4) + (lane >> 4);
    return *(const __attribute__((address_space(3))) hub_v4i *)(opb + row * HUB_K + ((c ^ (row & 7)) << 4));
}

// Patch number -> tile (ti <= tj) of an nb x nb tile grid; false when the
// patch or its tile lies outside the upper triangle.
__device__ inline bool hub_patch_tile(int nb, int patch, int within, int *ti, int *tj) {
    int pa_ = -1, pc_ = 0;
    int t = patch;
    for (int a = 0; a < hub_patch_rows(nb); a++) {
        const int c0 = (a * HUB_PR) / HUB_PC, cnt = hub_patch_cols(nb) - c0;
        if (t < cnt) { pa_ = a; pc_ = c0 + t; break; }
        t -= cnt;
    }
    *ti = pa_ * HUB_PR + within / HUB_PC;
    *tj = pc_ * HUB_PC + within % HUB_PC;
    return pa_ >= 0 && *ti < nb && *tj < nb && *ti <= *tj;
}

// One HUB_T x HUB_T tile (ti, tj) of Y Y^T over the kb bytes of the rows of
// y (row stride kb): HUB_WAVES waves in a 2 x (HUB_WAVES / 2) grid, each a
// 128 x HUB_WC part, 8 x HUB_BC products 16 x 16 x 128 (4-bit floats) per
// 64 bytes.
// Four waves of 128 x 128 would read a third less LDS per multiply-add
// (each fragment feeds eight products), but their 256 accumulators per
// lane make the compiler move accumulators between register files inside
// the loop: the wheel products took 10.1 s against 6.4 s with eight waves
// of 128 x 64 on the 4M-vertex graph, so eight it is.  Operands pass
// through two LDS buffers: the loads of the next step's bytes are in
// flight while the current step computes.  A step moves as many bytes
// through LDS (64 KB in, 192 KB of fragments out) as its products take
// cycles on the matrix cores; reading the second operand's fragments from
// memory into registers instead, one step ahead, cut that to 160 KB but
// left the products waiting on L2 (wheels 3.4 -> 5.8 s).  Every thread of
// the workgroup calls it.
__device__ inline void hub_tile(lds_u8 *lds, const uint8_t *y, int32_t kb, int ti, int tj,
                                hub_v4f (&cacc)[8][HUB_BC]) {
    const uint8_t *ya = y + (size_t)ti * HUB_T * kb, *yb = y + (size_t)tj * HUB_T * kb;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = (wid / (HUB_WAVES / 2)) * 128, wc = (wid % (HUB_WAVES / 2)) * HUB_WC;
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < HUB_BC; b++) cacc[a][b] = hub_v4f{0.f, 0.f, 0.f, 0.f};
    const int bufsz = 2 * HUB_T * HUB_K;
    hub_stage(lds, ya, yb, kb, 0, wid, lane);
    __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0): this wave's loads have landed
    __syncthreads();
    int cur = 0;
    for (int32_t k0 = 0; k0 < kb; k0 += HUB_K) {
        if (k0 + HUB_K < kb) hub_stage(lds + (cur ^ 1) * bufsz, ya, yb, kb, k0 + HUB_K, wid, lane);
        const lds_u8 *la = lds + cur * bufsz, *lb = la + HUB_T * HUB_K;
#pragma unroll
        for (int kk = 0; kk < HUB_K; kk += 64) {
            hub_v4i fa[8], fb[HUB_BC];
#pragma unroll
            for (int a = 0; a < 8; a++) fa[a] = hub_frag(la, wr + a * 16, kk, lane);
#pragma unroll
            for (int b = 0; b < HUB_BC; b++) fb[b] = hub_frag(lb, wc + b * 16, kk, lane);
#pragma unroll
            for (int a = 0; a < 8; a++)
#pragma unroll
                for (int b = 0; b < HUB_BC; b++)
                    cacc[a][b] = hub_mfma(fa[a], fb[b], cacc[a][b]);
        }
        // the next buffer has landed (every wave's part) and the current one
        // is read by every wave before it is loaded again
        __builtin_amdgcn_s_waitcnt(0xF70);
        __syncthreads();
        cur ^= 1;
    }
}

// Row i (within the tile, 0..HUB_T) and column j of accumulator element r of
// product (a, b) of this lane: result (r, c) of a 16 x 16 product sits in
// lane c + 16 * (r / 4), element r % 4.
__device__ inline int hub_acc_row(int wid, int lane, int a, int r) {
    return (wid / (HUB_WAVES / 2)) * 128 + a * 16 + 4 * (lane >> 4) + r;
}
__device__ inline int hub_acc_col(int wid, int lane, int b) { return (wid % (HUB_WAVES / 2)) * HUB_WC + b * 16 + (lane & 15); }

