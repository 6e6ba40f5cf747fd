// The bit-matrix encode on the matrix cores (gfx950 FP4 MFMA): the
// persistent kernels of the encode plans' form 2 and their launchers.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "gf_queue.h"
#include "gf_types.h"

namespace gfnc {

namespace {

// ------------------------------------------------------- encode, bit-matrix form
//
// Multiplication by a constant c is a GF(2)-linear map of a byte's 8 bits, an
// 8 x 8 bit matrix M_c, so a generation's encode is one GF(2) matrix product:
// (8K x 8N coefficient bits) x (8N x L source bits), each output bit the parity
// of a dot product of 0/1 values.  The matrix cores compute those dot products
// exactly: both operands are FP4 (E2M1) nibbles whose products are 0 or 1
// (fp4_source, fp4_coef), accumulation is FP32 from a bias of 2^23 (counts are
// exact integers in the low mantissa bits), and the parity is the lowest bit.
// The MFMA is the plain FP4 x FP4 form: zero scale arguments select the
// unscaled instruction.
//
// One MFMA 32x32x64: rows = 32 output bits (4 coded packets x 8 bits), columns
// = 32 payload bytes, reduction = 64 input bits (8 source packets x 8 bits).
// A workgroup tile is 16 coded packets (4 row tiles) over the whole packet in
// strips of 256 payload bytes; wave w covers 64 bytes of a strip (2 column
// tiles).  The coefficient operand of every step is built once per tile in LDS.

typedef int gf_v8i __attribute__((ext_vector_type(8)));
typedef float gf_v16f __attribute__((ext_vector_type(16)));

// FP4 (E2M1) operands whose values are 0 or a power of two.  A nibble with
// only bit 0, 1 or 2 set is 0.5, 1.0 or 2.0, so an operand register is a plain
// mask of the packed bits; bit 3 would be the sign, so bits 3 and 7 of a byte
// are shifted down first.  Register m of both operands holds the same two input
// bits of every byte (low nibble: bit j, high nibble: bit j + 4), and the two
// operands put them at nibble positions whose values multiply to exactly 1:
//   register   input bits   source operand   coefficient operand
//      0          0, 4         bit 0: 0.5         bit 2: 2.0
//      1          1, 5         bit 1: 1.0         bit 1: 1.0
//      2          2, 6         bit 2: 2.0         bit 0: 0.5
//      3          3, 7         bit 1: 1.0         bit 1: 1.0
// The coefficient operand is stored with bits 0 and 2 (and 4 and 6) of each
// byte swapped (coef_byte_order), so both sides are single masks; each
// product is 1 and the FP32 sum is the exact count of common set bits.
__device__ __forceinline__ gf_v8i fp4_source(uint32_t x)
{
    gf_v8i v;
    v[0] = (int)(x & 0x11111111u);
    v[1] = (int)(x & 0x22222222u);
    v[2] = (int)(x & 0x44444444u);
    v[3] = (int)((x >> 2) & 0x22222222u);
    v[4] = v[5] = v[6] = v[7] = 0;
    return v;
}

__device__ __forceinline__ gf_v8i fp4_coef(uint32_t y)
{
    gf_v8i v;
    v[0] = (int)(y & 0x44444444u);
    v[1] = (int)(y & 0x22222222u);
    v[2] = (int)(y & 0x11111111u);
    v[3] = (int)((y >> 2) & 0x22222222u);
    v[4] = v[5] = v[6] = v[7] = 0;
    return v;
}

// A bit-matrix row byte with bits 0 <-> 2 and 4 <-> 6 exchanged (see fp4_coef).
__device__ __forceinline__ uint8_t coef_byte_order(uint32_t b)
{
    return (uint8_t)((b & 0xAAu) | ((b & 0x11u) << 2) | ((b & 0x44u) >> 2));
}

// Bytes col and col + 1 of a row of len >= 1 bytes (zero past the end),
// without branches: the addresses are clamped into the row and the bytes
// outside it masked off, so a wave issues its loads back to back.  EVEN: the
// row start is 2-byte aligned and len >= 2 (one 16-bit load).
template <bool EVEN>
__device__ __forceinline__ uint32_t load_pair(const uint8_t *row, uint64_t col, uint64_t len)
{
    uint32_t v;
    if constexpr (EVEN) {
        const uint64_t c = col < len - 2 ? col : len - 2;
        v = *reinterpret_cast<const __attribute__((address_space(1))) uint16_t *>(
            reinterpret_cast<uintptr_t>(row + c));
        v = col + 1 == len ? v >> 8 : v;
    } else {
        const uint64_t c0 = col < len - 1 ? col : len - 1;
        const uint64_t c1 = col + 1 < len - 1 ? col + 1 : len - 1;
        const auto *gr = reinterpret_cast<const __attribute__((address_space(1))) uint8_t *>(
            reinterpret_cast<uintptr_t>(row));
        v = (uint32_t)gr[c0] | ((uint32_t)gr[c1] << 8);
    }
    v = col + 1 < len ? v : (v & 0xFFu);
    return col < len ? v : 0u;
}

// Row r of a 32-row tile of the coefficient-bit operand stands for coded
// packet 2*(r >> 4) + ((r >> 2) & 1) of the tile's four and for output bit
// 4*((r >> 3) & 1) + (r & 3).  With the 32x32 output layout of the matrix
// cores (lane c + 32h holds rows 8q + 4h + t, q, t < 4, as values 4q + t),
// lane c + 32h then holds all 8 bits of the output bytes of packets h and
// 2 + h at its column: values 8j .. 8j+7 are bits 0..7 of packet 2j + h.
__device__ __forceinline__ int mf_row_packet(int r) { return 2 * (r >> 4) + ((r >> 2) & 1); }
__device__ __forceinline__ int mf_row_bit(int r) { return 4 * ((r >> 3) & 1) + (r & 3); }

// Accumulators start at 2^23: a count c < 2^23 added to it is exact and sits in
// the low mantissa bits, so the count's parity is bit 0 of the float's bits.
constexpr float kParityBias = 8388608.0f;

// Parities of 8 biased counts -> one byte, bit u from v[base + u].
__device__ __forceinline__ uint32_t parity_byte(const gf_v16f &v, int base)
{
    uint32_t f[8];
#pragma unroll
    for (int u = 0; u < 8; u++)
        f[u] = __float_as_uint(v[base + u]);
    // low bytes of four floats side by side, then bit 0 of byte k moved to bit 24 + k
    const uint32_t w0 = __builtin_amdgcn_perm(f[1], f[0], 0x0c0c0400u) | __builtin_amdgcn_perm(f[3], f[2], 0x04000c0cu);
    const uint32_t w1 = __builtin_amdgcn_perm(f[5], f[4], 0x0c0c0400u) | __builtin_amdgcn_perm(f[7], f[6], 0x04000c0cu);
    const uint32_t lo = ((w0 & 0x01010101u) * 0x01020408u) >> 24;
    const uint32_t hi = ((w1 & 0x01010101u) * 0x01020408u) >> 24;
    return lo | (hi << 4);
}

// Tile set-up shared by the bit-matrix kernels: stage the tile's coefficient
// rows, then build the coefficient-bit operand for every step.  For lane
// (rr, hh) of row tile rt at step ks, byte s of Ybuf[ks][rt][lane] is row
// mf_row_bit(rr) of the bit matrix of C[k0 + 4 rt + mf_row_packet(rr)][8 ks +
// 4 hh + s], in coef_byte_order (TR holds the rows in that order).  Ends with
// a barrier.
__device__ __forceinline__ void mf_tile_setup(const DevGen &g, int k0, int nks, uint32_t (*Cl)[64],
                                              uint32_t (*Ybuf)[4][64], const uint8_t *TR, int tid)
{
    const int K = (int)g.K, N = (int)g.N, NP = nks * 8;
    uint8_t *Cb = reinterpret_cast<uint8_t *>(Cl);
    for (int e = tid; e < MF_ROWS * NP; e += 256) {
        const int pr = e / NP, n = e - pr * NP;
        Cb[pr * 256 + n] = (k0 + pr < K && n < N) ? g.C[(uint64_t)(k0 + pr) * N + n] : 0;
    }
    __syncthreads();
    for (int e = tid; e < nks * 256; e += 256) {
        const int ks = e >> 8, rt = (e >> 6) & 3, ln = e & 63;
        const int rr = ln & 31, hh = ln >> 5;
        const int pk = rt * 4 + mf_row_packet(rr), bit = mf_row_bit(rr);
        const uint32_t cw = Cl[pk][(ks * 8 + 4 * hh) >> 2];
        uint32_t Y = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
            Y |= (uint32_t)TR[((cw >> (8 * s)) & 0xFFu) * 8 + bit] << (8 * s);
        Ybuf[ks][rt][ln] = Y;
    }
    __syncthreads();
}

// Output bytes of one strip column pair (col, col + 1) of a wave: packets
// 2j + h of every row tile.  RUNNING: the accumulators hold a running total
// over the tile's strips, so this strip's parities are those of the total
// XOR those of the previous total, kept per lane in prev (two bytes per
// packet: prev[rt] holds j = 0 in bits 0..15 and j = 1 in bits 16..31).
// whole (wave-uniform): both columns of every lane lie inside the packet and
// the output rows are 2-byte aligned, so each packet's pair is one 16-bit store.
// Stores go through the global address space (no LDS counter traffic).
template <bool RUNNING>
__device__ __forceinline__ void mf_store(const DevGen &g, int k0, uint64_t col, gf_v16f (&acc)[4][2], int h,
                                         uint32_t (&prev)[4], bool whole)
{
    const int K = (int)g.K;
    uint32_t out[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        uint32_t pr = 0;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            uint32_t v = parity_byte(acc[rt][0], 8 * j) | (parity_byte(acc[rt][1], 8 * j) << 8);
            pr |= v << (16 * j);
            if (RUNNING)
                v ^= (prev[rt] >> (16 * j)) & 0xFFFFu;
            out[rt][j] = v;
        }
        if (RUNNING)
            prev[rt] = pr;
    }
    if (whole) {
        const uint8_t *base = g.Y + (uint64_t)(k0 + h) * g.ld_y + col;
#pragma unroll
        for (int rt = 0; rt < 4; rt++)
#pragma unroll
            for (int j = 0; j < 2; j++)
                if (k0 + 4 * rt + 2 * j + h < K)
                    *reinterpret_cast<__attribute__((address_space(1))) uint16_t *>(
                        reinterpret_cast<uintptr_t>(base + (uint64_t)(4 * rt + 2 * j) * g.ld_y)) =
                        (uint16_t)out[rt][j];
        return;
    }
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const uint32_t v = out[rt][j];
            const int row = k0 + 4 * rt + 2 * j + h;
            if (row >= K || col >= g.len)
                continue;
            auto *yp = reinterpret_cast<__attribute__((address_space(1))) uint8_t *>(
                reinterpret_cast<uintptr_t>(g.Y + (uint64_t)row * g.ld_y + col));
            if (col + 1 < g.len && ((reinterpret_cast<uintptr_t>(yp) & 1u) == 0)) {
                *reinterpret_cast<__attribute__((address_space(1))) uint16_t *>(yp) = (uint16_t)v;
            } else {
                yp[0] = (uint8_t)v;
                if (col + 1 < g.len)
                    yp[1] = (uint8_t)(v >> 8);
            }
        }
}

// Step ks of the product for one wave: 8 MFMAs over the 4 row tiles and 2
// column tiles; the first step of a strip starts from kParityBias.
__device__ __forceinline__ void mf_step(const uint32_t (*Ybuf)[4][64], int ks, int lane, uint32_t X0, uint32_t X1,
                                        gf_v16f (&acc)[4][2])
{
    const gf_v8i b0 = fp4_source(X0), b1 = fp4_source(X1);
    if (ks == 0) {
        gf_v16f bias;
#pragma unroll
        for (int v = 0; v < 16; v++)
            bias[v] = kParityBias;
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const gf_v8i a = fp4_coef(Ybuf[ks][rt][lane]);
            acc[rt][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b0, bias, 4, 4, 0, 0, 0, 0);
            acc[rt][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b1, bias, 4, 4, 0, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const gf_v8i a = fp4_coef(Ybuf[ks][rt][lane]);
            acc[rt][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b0, acc[rt][0], 4, 4, 0, 0, 0, 0);
            acc[rt][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b1, acc[rt][1], 4, 4, 0, 0, 0, 0);
        }
    }
}

// The strips of one tile for one wave: 64 payload bytes of every strip,
// all MF_ROWS coded rows, accumulating over the generation's sources 8 at a
// time; the source bytes of a step are loaded two steps ahead.
template <bool EVEN>
__device__ __forceinline__ void mf_tile(const DevGen &g, int k0, int nks, const uint32_t (*Ybuf)[4][64],
                                        gf_v16f (&acc)[4][2], int wave, int lane)
{
    const int r = lane & 31, h = lane >> 5;
    const int N = (int)g.N;
    const uint64_t nstrips = (g.len + MF_STRIP - 1) / MF_STRIP;
    const uint64_t lane_col = (uint64_t)wave * 64u + 2u * (uint64_t)r;
    auto load_src = [&](uint64_t strip, int ks, uint32_t (&u)[4]) {
        const uint64_t col = strip * MF_STRIP + lane_col;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int n = ks * 8 + 4 * h + s;
            const uint32_t v = load_pair<EVEN>(g.S + (uint64_t)(n < N ? n : N - 1) * g.ld_s, col, g.len);
            u[s] = (n < N && strip < nstrips) ? v : 0u;
        }
    };
    // prefetch position: (ps, pk) runs two steps ahead of (strip, ks)
    uint64_t ps = 0;
    int pk = 0;
    auto advance = [&]() {
        if (++pk == nks) {
            pk = 0;
            ps++;
        }
    };
    uint32_t cur[4], nxt[4], unused[4] = {};
    load_src(ps, pk, cur);
    advance();
    load_src(ps, pk, nxt);
    advance();
    for (uint64_t strip = 0; strip < nstrips; strip++) {
        for (int ks = 0; ks < nks; ks++) {
            const uint32_t t01 = __builtin_amdgcn_perm(cur[1], cur[0], 0x05010400u);
            const uint32_t t23 = __builtin_amdgcn_perm(cur[3], cur[2], 0x05010400u);
            const uint32_t X0 = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
            const uint32_t X1 = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
#pragma unroll
            for (int s = 0; s < 4; s++)
                cur[s] = nxt[s];
            load_src(ps, pk, nxt);
            advance();
            mf_step(Ybuf, ks, lane, X0, X1, acc);
        }
        mf_store<false>(g, k0, strip * MF_STRIP + lane_col, acc, h, unused, false);
    }
}

// Persistent: each workgroup takes tiles of MF_ROWS coded rows of one
// generation and runs over the whole packet length in strips of MF_STRIP
// bytes, so the coefficient-bit operand is built once per tile.
__global__ __launch_bounds__(256, GF_MF_WAVES_PER_SIMD) void k_encode_mfma(const DevGen *__restrict__ gens,
                                                                         const DevTile *__restrict__ tiles,
                                                                         const unsigned *__restrict__ runs,
                                                                         const unsigned *__restrict__ bounds,
                                                                         unsigned *counters,
                                                                         const uint8_t *__restrict__ rows_f)
{
    __shared__ uint8_t TR[256 * 8];
    __shared__ uint32_t Ybuf[256 / 8][4][64];   // coefficient bit rows per step, row tile and lane
    __shared__ uint32_t Cl[MF_ROWS][64];
    __shared__ int s_tile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 256 * 8; i += 256)
        TR[i] = coef_byte_order(rows_f[i]);
    gf_v16f acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 16; v++)
                acc[a][b][v] = 0.0f;

    QueueCursor cursor;
    for (;;) {
        if (tid == 0)
            s_tile = queue_next_tile(counters, runs, bounds, cursor);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t < 0)
            break;
        const DevTile tl = tiles[t];
        const DevGen g = gens[tl.gen];
        if (g.status && *g.status != g.need)
            continue;
        const int N = (int)g.N, k0 = (int)tl.k0;
        const int nks = (N + 7) >> 3;
        mf_tile_setup(g, k0, nks, Cl, Ybuf, TR, tid);
        // one instantiation only: two inlined copies sharing the accumulators
        // exhaust the register file, and byte loads cost little next to the MFMAs
        mf_tile<false>(g, k0, nks, Ybuf, acc, wave, lane);
    }
    if (tid == 0)
        queue_retire(counters, gridDim.x);
}

// Variant for sources whose row starts are 4-byte aligned: each wave copies
// its own source bytes of a step (8 rows x 64 bytes) into LDS through the load
// unit's direct-to-LDS path (4 bytes per lane, no registers), MF_STAGES - 1
// steps ahead of their use, so the waves of a workgroup never wait for one
// another inside a tile.  The steps of a tile (all strips, all source groups)
// form one software pipeline: while the matrix cores work on step z, the wave
// reads and unpacks the operands of step z + 1.
#ifndef GF_MF_STAGES
#define GF_MF_STAGES 8
#endif
constexpr int MF_STAGES = GF_MF_STAGES;
static_assert((MF_STAGES & (MF_STAGES - 1)) == 0 && MF_STAGES >= 2, "stages: a power of two");
// Steps come in pairs (two source groups of the same strip; a generation with
// an odd group count gets one zero group per strip), and a pair's sources are
// copied by four copy instructions, MF_PAIRS_AHEAD pairs ahead of the reads.
// A copy then only ever overwrites the slots of the previous pair, whose
// operands are in registers and used.  Every pair issues exactly four copies
// (past the tile's last step they copy a zero word), so when a step's operands
// are read the number of newer vector-memory loads in flight is known and one
// s_waitcnt vmcnt(n) is exact; in the gfx9 encoding vmcnt is bits 3:0 and 15:14,
// expcnt and lgkmcnt stay at their maxima (not waited for).  Stores issued in
// between only make a wait stricter: loads complete in order, so the count
// cannot drop that low while the awaited copy is pending.
constexpr int MF_PAIRS_AHEAD = MF_STAGES / 2 - 1;
static_assert(MF_PAIRS_AHEAD >= 1, "at least 4 stages");
constexpr int vm_wait(int newer_loads)
{
    return (newer_loads & 0xF) | ((newer_loads >> 4) << 14) | (0x7 << 4) | (0xF << 8);
}
constexpr int kWaitAll = vm_wait(0);
static_assert(4 * MF_PAIRS_AHEAD < 64, "vmcnt field is 6 bits");

// The operands of one step: the coefficient bits of the 4 row tiles and the
// source bits of the wave's 2 column tiles.
struct MfOperands {
    gf_v8i a[4];
    gf_v8i b[2];
};

template <int RT0 = 0, int RT1 = 4>
__device__ __forceinline__ void mf_mma(const MfOperands &o, gf_v16f (&acc)[4][2])
{
#pragma unroll
    for (int rt = RT0; rt < RT1; rt++) {
        acc[rt][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(o.a[rt], o.b[0], acc[rt][0], 4, 4, 0, 0, 0, 0);
        acc[rt][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(o.a[rt], o.b[1], acc[rt][1], 4, 4, 0, 0, 0, 0);
    }
}

constexpr int kMfRestart = 2048;

// Instruction order for the last NM products of a step and the unpacking of
// the next step's operands, one MFMA after every six vector instructions.
template <int NM>
__device__ __forceinline__ void mf_step_schedule()
{
#pragma unroll
    for (int i = 0; i < NM; i++) {
        __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);   // VALU
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    }
}

__device__ __forceinline__ void mf_acc_reset(gf_v16f (&acc)[4][2])
{
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 16; v++)
                acc[a][b][v] = kParityBias;
}

__global__ __launch_bounds__(256, GF_MF_WAVES_PER_SIMD) void k_encode_mfma_dma(const DevGen *__restrict__ gens,
                                                                             const DevTile *__restrict__ tiles,
                                                                             const unsigned *__restrict__ runs,
                                                                             const unsigned *__restrict__ bounds,
                                                                             unsigned *counters,
                                                                             const uint8_t *__restrict__ rows_f)
{
    __shared__ uint8_t TR[256 * 8];
    __shared__ uint32_t Ybuf[256 / 8][4][64];
    __shared__ uint32_t Cl[MF_ROWS][64];
    __shared__ uint32_t Sw[4][MF_STAGES][8][16];   // [wave][stage][source row][64 bytes]
    __shared__ int s_tile;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 31, h = lane >> 5;
    for (int i = tid; i < 256 * 8; i += 256)
        TR[i] = coef_byte_order(rows_f[i]);
    gf_v16f acc[4][2];

    QueueCursor cursor;
    for (;;) {
        if (tid == 0)
            s_tile = queue_next_tile(counters, runs, bounds, cursor);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t < 0)
            break;
        const DevTile tl = tiles[t];
        const DevGen g = gens[tl.gen];
        if (g.status && *g.status != g.need)
            continue;
        const int N = (int)g.N, k0 = (int)tl.k0;
        const int npairs = (N + 15) >> 4;       // pairs of 8-packet source groups
        const int nks = 2 * npairs;
        mf_tile_setup(g, k0, nks, Cl, Ybuf, TR, tid);
        const uint64_t ld = g.ld_s;
        const int nstrips = (int)((g.len + MF_STRIP - 1) / MF_STRIP);
        const int Zp = nstrips * npairs;        // the plan keeps this below 2^30
        // Copies of whole 16-row pairs inside whole strips are the generation's
        // source pointer plus a wave-uniform 32-bit offset plus a fixed per-lane
        // offset, when the generation's source span fits 31 bits.
        const int kp_full = N >> 4;
        const bool narrow = (uint64_t)N * ld + g.len < (1ull << 31);
        const bool y_even = ((reinterpret_cast<uintptr_t>(g.Y) | g.ld_y) & 1u) == 0;
        const int strips_full = narrow ? (int)(g.len / MF_STRIP) : 0;
        const uint32_t lcol = (uint32_t)wave * 64u + (uint32_t)(lane & 15) * 4u;
        const uint32_t ld4 = 4u * (uint32_t)ld;
        const uint32_t loff = (uint32_t)(lane >> 4) * (uint32_t)ld + lcol;
        // Copy cursor: pair cq = (strip cs, pair cp), whose first row starts
        // `coff` bytes into the source (valid while narrow; cbase for the rest).
        // Lane l copies 4 bytes of source rows 16 cp + l / 16 + {0, 4, 8, 12} at
        // byte (l % 16) * 4 of this wave's 64.  Outside the generation or the
        // packet a lane copies a zero word (row 0 of the table, the bit matrix
        // of 0): such bytes meet zero coefficient bits or are never stored.  A
        // chunk that straddles the packet end is assembled byte by byte (at most
        // 4 lanes per instruction).
        int cq = 0, cp = 0, cs = 0;
        uint32_t coff = 0, soff = 0;
        const uint8_t *cbase = g.S;
        auto copy_pair = [&]() {
            const int slot = (2 * cq) & (MF_STAGES - 1);
            if (cp < kp_full && cs < strips_full) {
#pragma unroll
                for (int q4 = 0; q4 < 4; q4++)
                    __builtin_amdgcn_global_load_lds(
                        reinterpret_cast<const void *>(g.S + (coff + loff + (uint32_t)q4 * ld4)),
                        (__attribute__((address_space(3))) void *)&Sw[wave][slot + (q4 >> 1)][4 * (q4 & 1)][0], 4,
                        0, 0);
            } else {
                const bool live = cq < Zp;
                const uint64_t rem = live ? g.len - (uint64_t)cs * MF_STRIP : 0;
                const int remrows = live ? N - cp * 16 : 0;
#pragma unroll
                for (int q4 = 0; q4 < 4; q4++) {
                    const int rr = 4 * q4 + (lane >> 4);
                    const uint8_t *src = cbase + (uint64_t)rr * ld + lcol;
                    uint32_t *dst = &Sw[wave][slot + (q4 >> 1)][4 * (q4 & 1)][0];
                    const bool rowok = rr < remrows;
                    const bool full = rowok && lcol + 4 <= rem;
                    const bool straddle = rowok && lcol < rem && !full;
                    if (!straddle) {
                        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(full ? src : rows_f),
                                                         (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
                    } else {
                        uint32_t v = 0;
                        for (uint32_t b = 0; lcol + b < rem; b++)
                            v |= (uint32_t)src[b] << (8 * b);
                        dst[lane] = v;
                    }
                }
            }
            cq++;
            if (++cp == npairs) {
                cp = 0;
                cs++;
                soff += MF_STRIP;
                coff = soff;
                cbase = g.S + (uint64_t)cs * MF_STRIP;
            } else {
                coff += 16u * (uint32_t)ld;
                cbase += 16u * ld;
            }
        };
        // Operands of step zf (source group ksf), in two parts: fetch_issue
        // waits until the step's copy has landed (once the newer copies alone
        // are outstanding) and issues the LDS reads; fetch_unpack builds the
        // MFMA operands.  Bytes of rows past N and past the packet end need no
        // masking (see copy_pair).
        struct Raw {
            uint32_t s[4];   // columns 2r, 2r + 1 of source rows 0..3 (one 16-bit read each)
            uint32_t y[4];
        };
        // A tile's last 16 coded rows may be fewer: only the row tiles (of 4
        // packets) that hold rows of the generation are multiplied (RTS).
        const int rts = min(4, ((int)g.K - k0 + 3) >> 2);
        auto run_tile = [&](auto rts_c) {
        constexpr int RTS = decltype(rts_c)::value;
        auto fetch_issue = [&](int zf, int ksf, auto wait_imm) {
            __builtin_amdgcn_s_waitcnt(decltype(wait_imm)::value);
            asm volatile("" ::: "memory");
            const uint16_t *rows = reinterpret_cast<const uint16_t *>(&Sw[wave][zf & (MF_STAGES - 1)][4 * h][0]);
            Raw w;
#pragma unroll
            for (int q = 0; q < 4; q++)
                w.s[q] = rows[q * 32 + r];
#pragma unroll
            for (int rt = 0; rt < RTS; rt++)
                w.y[rt] = Ybuf[ksf][rt][lane];
            return w;
        };
        auto fetch_unpack = [&](const Raw &w, MfOperands &o) {
            const uint32_t t01 = __builtin_amdgcn_perm(w.s[1], w.s[0], 0x05010400u);   // r0c0 r1c0 r0c1 r1c1
            const uint32_t t23 = __builtin_amdgcn_perm(w.s[3], w.s[2], 0x05010400u);   // r2c0 r3c0 r2c1 r3c1
            o.b[0] = fp4_source(__builtin_amdgcn_perm(t23, t01, 0x05040100u));   // column 2r of rows 0..3
            o.b[1] = fp4_source(__builtin_amdgcn_perm(t23, t01, 0x07060302u));   // column 2r + 1
#pragma unroll
            for (int rt = 0; rt < RTS; rt++)
                o.a[rt] = fp4_coef(w.y[rt]);
        };
        // One step: the next operands are read and unpacked while this step's
        // products run.  The fences keep the LDS reads first and the first two
        // products next, so the wait for the reads (the reads are kept as four
        // separate words, since packing them would need their values at once)
        // sits behind two MFMAs instead of in front of them.
        // MMA false: this step's sources are the zero group that pads an odd
        // group count, so only the next operands are fetched.
        auto step = [&](int zn, int ksn, const MfOperands &cur, MfOperands &nxt, auto wait_imm, auto mma_c) {
            const Raw w = fetch_issue(zn, ksn, wait_imm);
            if constexpr (decltype(mma_c)::value) {
                __builtin_amdgcn_sched_barrier(0);
                mf_mma<0, 1>(cur, acc);
                __builtin_amdgcn_sched_barrier(0);
                fetch_unpack(w, nxt);
                mf_mma<1, RTS>(cur, acc);
                mf_step_schedule<2 * RTS - 2>();
            } else {
                fetch_unpack(w, nxt);
            }
        };
        using Mma = std::true_type;
        using NoMma = std::false_type;
        const bool odd_groups = ((N + 7) >> 3) & 1;   // the last step of each strip multiplies zeros

        // Before the pair starting at step z = 2q, copies are issued through
        // pair q + MF_PAIRS_AHEAD - 1.  Reading step 2q + 1 (after this pair's
        // copies): 4 MF_PAIRS_AHEAD newer loads; reading step 2q + 2: 2 fewer.
        using WaitOdd = std::integral_constant<int, vm_wait(4 * MF_PAIRS_AHEAD)>;
        using WaitEven = std::integral_constant<int, vm_wait(4 * MF_PAIRS_AHEAD - 2)>;
        for (int j = 0; j < MF_PAIRS_AHEAD; j++)
            copy_pair();
        mf_acc_reset(acc);
        // Two operand sets take turns, so no registers are copied between steps.
        MfOperands opa, opb;
        fetch_unpack(fetch_issue(0, 0, WaitEven{}), opa);
        // The accumulators run over all strips of the tile and restart every
        // kMfRestart strips: a strip adds at most 64 nks <= 2048 to a count, so
        // the total stays below 2^23 + 2^22, exact in FP32.
        uint32_t prev[4] = {0u, 0u, 0u, 0u};
        int z = 0;
        for (int strip = 0; strip < nstrips; strip++) {
            for (int kp = 0; kp + 1 < npairs; kp++, z += 2) {
                copy_pair();              // pair q + MF_PAIRS_AHEAD, into the slots of pair q - 1
                step(z + 1, 2 * kp + 1, opa, opb, WaitOdd{}, Mma{});
                step(z + 2, 2 * kp + 2, opb, opa, WaitEven{}, Mma{});
            }
            // the strip's last pair; its second step fetches the next strip's first (past the end: a zero slot)
            copy_pair();
            step(z + 1, nks - 1, opa, opb, WaitOdd{}, Mma{});
            if (odd_groups)
                step(z + 2, 0, opb, opa, WaitEven{}, NoMma{});
            else
                step(z + 2, 0, opb, opa, WaitEven{}, Mma{});
            z += 2;
            mf_store<true>(g, k0, (uint64_t)strip * MF_STRIP + (uint64_t)wave * 64u + 2u * (uint64_t)r, acc, h,
                           prev, y_even && (uint64_t)(strip + 1) * MF_STRIP <= g.len);
            if ((strip & (kMfRestart - 1)) == kMfRestart - 1) {
                mf_acc_reset(acc);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    prev[i] = 0u;
            }
        }
        };
        if (rts >= 4)
            run_tile(std::integral_constant<int, 4>{});
        else if (rts == 3)
            run_tile(std::integral_constant<int, 3>{});
        else if (rts == 2)
            run_tile(std::integral_constant<int, 2>{});
        else
            run_tile(std::integral_constant<int, 1>{});
        // the copies past the last step land before the slots are reused
        __builtin_amdgcn_s_waitcnt(kWaitAll);
        __syncthreads();   // every wave is done with Cl and Ybuf before the next tile
    }
    if (tid == 0)
        queue_retire(counters, gridDim.x);
}

}  // namespace

// ----------------------------------------------------------------- launchers

hipError_t launch_encode_mfma(const DevGen *gens, const DevTile *tiles, const unsigned *runs, const unsigned *bounds,
                              int ntiles, unsigned *counters, int grid, const uint8_t *rows_field, bool aligned4,
                              hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (aligned4)
        hipLaunchKernelGGL(k_encode_mfma_dma, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters,
                           rows_field);
    else
        hipLaunchKernelGGL(k_encode_mfma, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters,
                           rows_field);
    return hipGetLastError();
}

int encode_mfma_blocks_per_cu(bool aligned4)
{
    // the same for every gfx950 device; asked once (launches may be under graph capture)
    static int cached[2] = {0, 0};
    int &nb = cached[aligned4 ? 1 : 0];
    if (nb > 0)
        return nb;
    int v = 0;
    const void *k = aligned4 ? reinterpret_cast<const void *>(&k_encode_mfma_dma)
                              : reinterpret_cast<const void *>(&k_encode_mfma);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k, 256, 0) != hipSuccess || v < 1)
        return 1;
    nb = v;
    return nb;
}

}  // namespace gfnc
