// HIP kernels for GF(2^n) network coding on gfx950 (CDNA4).
//
// Arithmetic.  Multiplying a byte of packed words by a field constant c is a
// GF(2)-linear map of the byte's 8 bits, so c*b = c*(b & 0x07) ^ c*(b & 0x38)
// ^ c*(b & 0xC0).  Each of the three parts takes at most 8 values, which is
// exactly what one V_PERM_B32 byte-select can look up: it picks, for each of
// the 4 bytes of a dword, one of 8 bytes held in two registers.  Three perms
// and two XORs therefore multiply 4 payload bytes by c.  This is the paper's
// table-lookup ("shuffle", Sec. IV-A, Algorithm 1) idea -- per-coefficient
// product tables indexed by pieces of the data byte -- resized to the 8-entry
// byte select that CDNA provides in place of a 16-entry byte shuffle.  The
// same tables serve GF(2), GF(4), GF(16) and GF(256) because the product is
// applied word by word inside the byte.
//
// Encode (Sec. II, Eq. 1, for K coding vectors) keeps KW coded rows of a
// payload strip in registers and streams the N source rows through them once;
// the per-(row, source) tables are staged in LDS and read with wave-uniform
// addresses (broadcast, no bank conflicts).
#include <algorithm>
#include <type_traits>

#include "gf_internal.h"

namespace gfnc {

namespace {

constexpr int NC = 32;   // source rows per LDS table stage

struct Sel {
    uint32_t a, b, c;
};

__device__ __forceinline__ Sel split(uint32_t x)
{
    Sel s;
    s.a = x & 0x07070707u;
    s.b = (x >> 3) & 0x07070707u;
    s.c = (x >> 6) & 0x03030303u;
    return s;
}

// Product of the 4 bytes behind `s` with the coefficient whose tables are
// (t0,t1) for bits 0-2, (t2,t3) for bits 3-5 and t4 for bits 6-7.
__device__ __forceinline__ uint32_t prod(uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3, uint32_t t4,
                                         const Sel &s)
{
    return __builtin_amdgcn_perm(t1, t0, s.a) ^ __builtin_amdgcn_perm(t3, t2, s.b) ^
           __builtin_amdgcn_perm(t4, t4, s.c);
}

__device__ __forceinline__ uint32_t prod4(const uint4 &ta, uint32_t tb, uint32_t x)
{
    return prod(ta.x, ta.y, ta.z, ta.w, tb, split(x));
}

// Plain loads and stores through the global address space: a generic (flat)
// access also counts against the LDS wait counter, so an LDS read issued
// after it would wait for the global load as well and undo the prefetch.
typedef uint32_t gf_u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t gf_u32x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ T gld(const void *p)
{
    return *reinterpret_cast<const __attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p));
}

template <class T>
__device__ __forceinline__ void gst(void *p, T v)
{
    *reinterpret_cast<__attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p)) = v;
}

template <int D>
__device__ __forceinline__ void load_row(const uint8_t *p, uint64_t avail, bool vec, uint32_t (&x)[D])
{
    if (vec && avail >= 4u * D) {
        if constexpr (D == 4) {
            const gf_u32x4 t = gld<gf_u32x4>(p);
            x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
        } else if constexpr (D == 2) {
            const gf_u32x2 t = gld<gf_u32x2>(p);
            x[0] = t.x; x[1] = t.y;
        } else {
            x[0] = gld<uint32_t>(p);
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; d++)
            x[d] = 0;
#pragma unroll
        for (int b = 0; b < 4 * D; b++)
            if ((uint64_t)b < avail)
                x[b >> 2] |= (uint32_t)gld<uint8_t>(p + b) << (8 * (b & 3));
    }
}

template <int D>
__device__ __forceinline__ void store_row(uint8_t *p, uint64_t avail, bool vec, const uint32_t (&x)[D])
{
    if (vec && avail >= 4u * D) {
        if constexpr (D == 4) {
            gst<gf_u32x4>(p, gf_u32x4{x[0], x[1], x[2], x[3]});
        } else if constexpr (D == 2) {
            gst<gf_u32x2>(p, gf_u32x2{x[0], x[1]});
        } else {
            gst<uint32_t>(p, x[0]);
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4 * D; b++)
            if ((uint64_t)b < avail)
                gst<uint8_t>(p + b, (uint8_t)(x[b >> 2] >> (8 * (b & 3))));
    }
}

// ------------------------------------------------------------------ region

// mode 0: y ^= c*x (madd);  mode 1: y = c*x.
// Bytes [0, head) and the tail go byte by byte; the middle in 16-byte vectors
// when x and y share their offset modulo 16 (vec != 0).
template <int MODE>
__global__ __launch_bounds__(256) void k_region(uint8_t *y, const uint8_t *x, uint64_t len, uint32_t t0,
                                                uint32_t t1, uint32_t t2, uint32_t t3, uint32_t t4, int vec)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t head = 0, nvec = 0;
    if (vec) {
        head = (16u - ((uintptr_t)y & 15u)) & 15u;
        if (head > len)
            head = len;
        nvec = (len - head) >> 4;
    }
    const uint4 *xv = reinterpret_cast<const uint4 *>(x + head);
    uint4 *yv = reinterpret_cast<uint4 *>(y + head);
    uint64_t i = gid;
    for (; i + stride < nvec; i += 2 * stride) {
        const uint4 a = xv[i], b = xv[i + stride];
        uint4 ra, rb;
        ra.x = prod(t0, t1, t2, t3, t4, split(a.x));
        ra.y = prod(t0, t1, t2, t3, t4, split(a.y));
        ra.z = prod(t0, t1, t2, t3, t4, split(a.z));
        ra.w = prod(t0, t1, t2, t3, t4, split(a.w));
        rb.x = prod(t0, t1, t2, t3, t4, split(b.x));
        rb.y = prod(t0, t1, t2, t3, t4, split(b.y));
        rb.z = prod(t0, t1, t2, t3, t4, split(b.z));
        rb.w = prod(t0, t1, t2, t3, t4, split(b.w));
        if (MODE == 0) {
            const uint4 ya = yv[i], yb = yv[i + stride];
            ra.x ^= ya.x; ra.y ^= ya.y; ra.z ^= ya.z; ra.w ^= ya.w;
            rb.x ^= yb.x; rb.y ^= yb.y; rb.z ^= yb.z; rb.w ^= yb.w;
        }
        yv[i] = ra;
        yv[i + stride] = rb;
    }
    for (; i < nvec; i += stride) {
        const uint4 a = xv[i];
        uint4 r;
        r.x = prod(t0, t1, t2, t3, t4, split(a.x));
        r.y = prod(t0, t1, t2, t3, t4, split(a.y));
        r.z = prod(t0, t1, t2, t3, t4, split(a.z));
        r.w = prod(t0, t1, t2, t3, t4, split(a.w));
        if (MODE == 0) {
            const uint4 ya = yv[i];
            r.x ^= ya.x; r.y ^= ya.y; r.z ^= ya.z; r.w ^= ya.w;
        }
        yv[i] = r;
    }
    // bytes outside the vector body: [0, head) and [head + 16*nvec, len)
    const uint64_t body_end = head + (nvec << 4);
    const uint64_t rest = head + (len - body_end);
    for (uint64_t j = gid; j < rest; j += stride) {
        const uint64_t b = j < head ? j : body_end + (j - head);
        const uint32_t pr = prod(t0, t1, t2, t3, t4, split((uint32_t)x[b])) & 0xFFu;
        y[b] = (uint8_t)(MODE == 0 ? (y[b] ^ pr) : pr);
    }
}

struct RegionDesc {
    uint8_t *y;
    const uint8_t *x;
    uint64_t len;
    uint32_t c;
    uint32_t reserved;
};

constexpr int REGION_CHUNK = 256 * 16;   // bytes per block per region

// Batched madd: block (bx, r) handles bytes [bx*REGION_CHUNK, ...) of region r.
__global__ __launch_bounds__(256) void k_region_batched(const RegionDesc *__restrict__ regs,
                                                        const uint4 *__restrict__ ptab4, int q)
{
    const RegionDesc d = regs[blockIdx.y];
    const uint64_t start = (uint64_t)blockIdx.x * REGION_CHUNK;
    if (d.c == 0 || d.c >= (uint32_t)q || start >= d.len)
        return;
    const uint4 ta = ptab4[d.c * 2];
    const uint32_t tb = ptab4[d.c * 2 + 1].x;
    const uint64_t end = min(d.len, start + REGION_CHUNK);
    const bool vec = (((uintptr_t)d.y | (uintptr_t)d.x) & 15u) == 0;
    const uint64_t p = start + threadIdx.x * 16u;
    if (vec && p + 16 <= end) {
        const uint4 a = *reinterpret_cast<const uint4 *>(d.x + p);
        uint4 yv = *reinterpret_cast<const uint4 *>(d.y + p);
        yv.x ^= prod4(ta, tb, a.x);
        yv.y ^= prod4(ta, tb, a.y);
        yv.z ^= prod4(ta, tb, a.z);
        yv.w ^= prod4(ta, tb, a.w);
        *reinterpret_cast<uint4 *>(d.y + p) = yv;
    } else if (p < end) {
        for (uint64_t b = p; b < min(end, p + 16); b++)
            d.y[b] ^= (uint8_t)(prod4(ta, tb, (uint32_t)d.x[b]) & 0xFFu);
    }
}

// ------------------------------------------------------------------ encode

constexpr int KW = ENC_ROWS;   // coded rows per wave tile
constexpr int NCW = 8;     // source rows per table stage (even)
constexpr int WAVES = 4;   // waves per workgroup

// One wave's staged product tables: [coded row][source row][2 x uint4].
struct WaveStage {
    uint4 t[KW][NCW][2];
};

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wavefront complete in order; this only keeps the
    // compiler from moving LDS accesses across the stage boundary.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

template <int D>
__device__ __forceinline__ void load_lane(const uint8_t *p, uint64_t avail, bool vec, uint32_t (&x)[D])
{
    if (avail == 0) {
#pragma unroll
        for (int d = 0; d < D; d++)
            x[d] = 0;
    } else {
        load_row<D>(p, avail, vec, x);
    }
}

// One wave tile: coded rows k0 .. k0+min(KW, K-k0)-1 over the 256*D payload
// bytes starting at p0 (4*D bytes per lane).  The N source rows stream
// through in pairs; each coded row accumulates, per dword of 4 bytes, the
// three byte-select products of both sources with two 3-input XORs.
// staged: the wave's stage already holds the tables of sources nb .. ne-1
// (ne - nb <= NCW, the same rows and sources as a previous call).
template <int D>
__device__ __forceinline__ void wave_tile(const uint8_t *__restrict__ C, int K, int N,
                                          const uint8_t *__restrict__ S, uint64_t ld_s, uint8_t *__restrict__ Y,
                                          uint64_t ld_y, uint64_t len, int k0, uint64_t p0, bool vec,
                                          const uint4 *__restrict__ ptab4, WaveStage &st, int lane, int nb, int ne,
                                          bool atomic_out, bool staged = false)
{
    const uint64_t p = p0 + (uint64_t)lane * (4u * D);
    const uint64_t avail = p < len ? len - p : 0;
    const int kv = min(KW, K - k0);

    uint32_t acc[KW][D];
#pragma unroll
    for (int kk = 0; kk < KW; kk++)
#pragma unroll
        for (int d = 0; d < D; d++)
            acc[kk][d] = 0;

    const uint8_t *src = S + p;
    uint32_t xa[D], xb[D];
    load_lane<D>(src + (uint64_t)nb * ld_s, avail, vec, xa);
    if (nb + 1 < ne)
        load_lane<D>(src + (uint64_t)(nb + 1) * ld_s, avail, vec, xb);
    else
#pragma unroll
        for (int d = 0; d < D; d++)
            xb[d] = 0;

    for (int g = nb; g < ne; g += 2) {
        const int nn = (g - nb) & (NCW - 1);
        if (nn == 0 && !staged) {
            wave_sync();
            const int nc = min(NCW, ne - g);
#pragma unroll
            for (int e = lane; e < KW * NCW; e += 64) {
                const int kk = e / NCW, j = e % NCW;
                const uint32_t c = (kk < kv && j < nc) ? (uint32_t)gld<uint8_t>(C + (uint64_t)(k0 + kk) * N + g + j) : 0u;
                st.t[kk][j][0] = ptab4[c * 2];
                st.t[kk][j][1] = ptab4[c * 2 + 1];
            }
            wave_sync();
        }
        Sel sa[D], sb[D];
#pragma unroll
        for (int d = 0; d < D; d++) {
            sa[d] = split(xa[d]);
            sb[d] = split(xb[d]);
        }
        const bool two = g + 1 < ne;
        if (g + 2 < ne)
            load_lane<D>(src + (uint64_t)(g + 2) * ld_s, avail, vec, xa);
        if (g + 3 < ne)
            load_lane<D>(src + (uint64_t)(g + 3) * ld_s, avail, vec, xb);
        if (two) {
#pragma unroll
            for (int k8 = 0; k8 < KW; k8 += 8) {
                if (k8 < kv) {
#pragma unroll
                    for (int kk = k8; kk < k8 + 8; kk++) {
                        const uint4 a0 = st.t[kk][nn][0];
                        const uint32_t b0 = st.t[kk][nn][1].x;
                        const uint4 a1 = st.t[kk][nn + 1][0];
                        const uint32_t b1 = st.t[kk][nn + 1][1].x;
#pragma unroll
                        for (int d = 0; d < D; d++) {
                            const uint32_t p0_ = __builtin_amdgcn_perm(a0.y, a0.x, sa[d].a);
                            const uint32_t p1_ = __builtin_amdgcn_perm(a0.w, a0.z, sa[d].b);
                            const uint32_t p2_ = __builtin_amdgcn_perm(b0, b0, sa[d].c);
                            const uint32_t q0_ = __builtin_amdgcn_perm(a1.y, a1.x, sb[d].a);
                            const uint32_t q1_ = __builtin_amdgcn_perm(a1.w, a1.z, sb[d].b);
                            const uint32_t q2_ = __builtin_amdgcn_perm(b1, b1, sb[d].c);
                            acc[kk][d] = xor3(xor3(xor3(acc[kk][d], p0_, p1_), p2_, q0_), q1_, q2_);
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int k8 = 0; k8 < KW; k8 += 8) {
                if (k8 < kv) {
#pragma unroll
                    for (int kk = k8; kk < k8 + 8; kk++) {
                        const uint4 a0 = st.t[kk][nn][0];
                        const uint32_t b0 = st.t[kk][nn][1].x;
#pragma unroll
                        for (int d = 0; d < D; d++) {
                            const uint32_t p0_ = __builtin_amdgcn_perm(a0.y, a0.x, sa[d].a);
                            const uint32_t p1_ = __builtin_amdgcn_perm(a0.w, a0.z, sa[d].b);
                            const uint32_t p2_ = __builtin_amdgcn_perm(b0, b0, sa[d].c);
                            acc[kk][d] = xor3(acc[kk][d], p0_, p1_) ^ p2_;
                        }
                    }
                }
            }
        }
    }
    if (avail == 0)
        return;
    if (atomic_out) {
        // Partial sum over a slice of the sources: XOR it into the zeroed
        // output.  Rows are 4-byte aligned here; only whole dwords below
        // len & ~3 are written (the last 0-3 bytes of each row are computed
        // by k_encode_tail).
        const uint64_t len4 = len & ~(uint64_t)3;
#pragma unroll
        for (int kk = 0; kk < KW; kk++)
            if (kk < kv) {
                uint32_t *yp = reinterpret_cast<uint32_t *>(Y + (uint64_t)(k0 + kk) * ld_y + p);
#pragma unroll
                for (int d = 0; d < D; d++)
                    if (p + 4u * d + 4u <= len4)
                        atomicXor(yp + d, acc[kk][d]);
            }
        return;
    }
#pragma unroll
    for (int kk = 0; kk < KW; kk++)
        if (kk < kv)
            store_row<D>(Y + (uint64_t)(k0 + kk) * ld_y + p, avail, vec, acc[kk]);
}

// Single generation: wave w of block b takes tile b*WAVES + w; tiles run
// over payload strips of 256*D bytes, then over `nsplit` slices of the
// sources (each slice's partial sum is XORed into a zeroed output), then over
// blocks of KW coded rows.
template <int D>
__global__ __launch_bounds__(256, GF_ENC_WAVES_PER_SIMD) void k_encode_direct(
    const uint8_t *__restrict__ C, int K, int N, const uint8_t *__restrict__ S, uint64_t ld_s,
    uint8_t *__restrict__ Y, uint64_t ld_y, uint64_t len, const uint4 *__restrict__ ptab4,
    const int *__restrict__ status, int need, int vec, uint32_t nstrips, uint32_t nsplit, uint32_t ntiles)
{
    __shared__ WaveStage stage[WAVES];
    if (status && *status != need)
        return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t t = blockIdx.x * WAVES + wave;
    if (t >= ntiles)
        return;
    const uint32_t strip = t % nstrips;
    const uint32_t rest = t / nstrips;
    const uint32_t sl = rest % nsplit, kb = rest / nsplit;
    const int chunk = (((N + (int)nsplit - 1) / (int)nsplit) + 1) & ~1;
    const int nb = (int)sl * chunk, ne = min(N, nb + chunk);
    if (nb >= ne)
        return;
    wave_tile<D>(C, K, N, S, ld_s, Y, ld_y, len, (int)(kb * KW), (uint64_t)strip * (256u * D), vec != 0, ptab4,
                 stage[wave], lane, nb, ne, nsplit > 1);
}

// The last len % 4 bytes of every coded row, each computed in full by one
// thread (used with the source-sliced launch, whose atomics cover whole dwords).
__global__ __launch_bounds__(256) void k_encode_tail(const uint8_t *__restrict__ C, int K, int N,
                                                     const uint8_t *__restrict__ S, uint64_t ld_s,
                                                     uint8_t *__restrict__ Y, uint64_t ld_y, uint64_t len,
                                                     const uint4 *__restrict__ ptab4,
                                                     const int *__restrict__ status, int need)
{
    if (status && *status != need)
        return;
    const int tail = (int)(len & 3);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * tail)
        return;
    const int k = i / tail;
    const uint64_t b = (len & ~(uint64_t)3) + (uint64_t)(i - k * tail);
    uint32_t acc = 0;
    for (int n = 0; n < N; n++) {
        const uint32_t c = C[(uint64_t)k * N + n];
        acc ^= prod4(ptab4[c * 2], ptab4[c * 2 + 1].x, (uint32_t)S[(uint64_t)n * ld_s + b]);
    }
    Y[(uint64_t)k * ld_y + b] = (uint8_t)acc;
}

// Y rows := 0 up to len & ~3 (before a launch that accumulates source slices
// atomically).
__global__ __launch_bounds__(256) void k_zero_rows(uint8_t *Y, uint64_t ld_y, uint64_t len, int K,
                                                   const int *__restrict__ status, int need)
{
    if (status && *status != need)
        return;
    const uint64_t words = len / 4;
    const uint64_t total = words * (uint64_t)K;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = i / words, w = i - k * words;
        reinterpret_cast<uint32_t *>(Y + k * ld_y)[w] = 0;
    }
}

// ---------------------------------------------------------------- work queues
// (layout of runs, bounds and counters: see TileQueues)

// Next run for a workgroup or wave (one lane calls), or -1 when every queue
// is empty: the home queue of this workgroup's XCD first, then the others in
// turn; q counts the queues found empty so far.
__device__ __forceinline__ int queue_take_run(unsigned *counters, const unsigned *__restrict__ bounds, int &q)
{
    const int home = (int)(blockIdx.x % MF_QUEUES);
    while (q < MF_QUEUES) {
        const int qi = (home + q) % MF_QUEUES;
        const unsigned lo = bounds[qi], hi = bounds[qi + 1];
        if (lo < hi) {
            const unsigned t = atomicAdd(&counters[MF_CTR_STRIDE * qi], 1u);
            if (t < hi - lo)
                return (int)(lo + t);
        }
        q++;
    }
    return -1;
}

// Tile cursor of a claimant: the rest of its current run, then the next run.
struct QueueCursor {
    int q = 0;
    unsigned next = 0, end = 0;
};

__device__ __forceinline__ int queue_next_tile(unsigned *counters, const unsigned *__restrict__ runs,
                                               const unsigned *__restrict__ bounds, QueueCursor &c)
{
    while (c.next == c.end) {
        const int r = queue_take_run(counters, bounds, c.q);
        if (r < 0)
            return -1;
        c.next = runs[r];
        c.end = runs[r + 1];
    }
    return (int)c.next++;
}

// The last of `claimants` to finish sets every counter back to zero.
__device__ __forceinline__ void queue_retire(unsigned *counters, unsigned claimants)
{
    __threadfence();
    if (atomicAdd(&counters[MF_CTR_RETIRED], 1u) == claimants - 1) {
        for (int i = 0; i < MF_QUEUES; i++)
            atomicExch(&counters[MF_CTR_STRIDE * i], 0u);
        atomicExch(&counters[MF_CTR_RETIRED], 0u);
    }
}

// Persistent encode over the work queues; every wave claims tiles on its own.
__global__ __launch_bounds__(256, GF_ENC_WAVES_PER_SIMD) void k_encode_waves(const DevGen *__restrict__ gens,
                                                      const DevTile *__restrict__ tiles,
                                                      const unsigned *__restrict__ runs,
                                                      const unsigned *__restrict__ bounds, unsigned *counters,
                                                      const uint4 *__restrict__ ptab4)
{
    __shared__ WaveStage stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    QueueCursor cursor;
    for (;;) {
        int t = 0;
        if (lane == 0)
            t = queue_next_tile(counters, runs, bounds, cursor);
        t = __builtin_amdgcn_readlane(t, 0);
        if (t < 0)
            break;
        const DevTile tl = tiles[t];
        const DevGen g = gens[tl.gen];
        if (g.status && *g.status != g.need)
            continue;
        // strips after the first reuse the staged tables when one stage holds every source
        const int d = tl.D & 0xFF, strips = (tl.D >> 8) + 1;
        for (int q = 0; q < strips; q++) {
            const uint64_t p0 = tl.p0 + (uint64_t)q * 256u * (uint64_t)d;
            const bool staged = q > 0 && (int)g.N <= NCW;
            if (d == 4)
                wave_tile<4>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                             g.align >= 16, ptab4, stage[wave], lane, 0, (int)g.N, false, staged);
            else if (d == 2)
                wave_tile<2>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                             g.align >= 8, ptab4, stage[wave], lane, 0, (int)g.N, false, staged);
            else
                wave_tile<1>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                             g.align >= 4, ptab4, stage[wave], lane, 0, (int)g.N, false, staged);
        }
    }
    if (lane == 0)
        queue_retire(counters, gridDim.x * WAVES);
}

// ------------------------------------------------------- encode, bit-plane form
//
// For n <= 4 a product is cheapest as the XOR of bit planes: with c = sum of
// c_b alpha^b, c * x = XOR over b of c_b (alpha^b x), and alpha^b x is a few
// shifts and masks of the packed words (the GF(2)-linearity behind the
// paper's Alg. 2, with the coefficient split into bits instead of the data).
// The planes of a source dword are built once and shared by every coded row
// of the tile; each (row, source, plane) then costs one 3-input bit operation
// per dword, acc ^ (plane & mask), where mask is all ones when bit b of the
// coefficient is set.  The masks are staged in LDS per wave, the two sources
// of a step side by side, so one uniform LDS read serves 2 n of them.

// a ^ (b & c) in one instruction (truth table over src0 = 0xF0, src1 = 0xCC,
// src2 = 0xAA); written out so the compiler keeps one per (row, source, plane)
// instead of regrouping the XORs.
__device__ __forceinline__ uint32_t and_xor(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x78);
}

// x times alpha for every n-bit word of x.
template <int NB>
__device__ __forceinline__ uint32_t times_alpha(uint32_t x)
{
    if constexpr (NB == 2) {
        // x^2 = x + 1: (h, l) -> (h ^ l, h)
        return ((x >> 1) & 0x55555555u) | ((x ^ (x << 1)) & 0xAAAAAAAAu);
    } else {
        // x^4 = x + 1: shift up within the nibble, the top bit folds into bits 0 and 1
        const uint32_t t = x & 0x88888888u;
        return ((x << 1) & 0xEEEEEEEEu) ^ (t >> 3) ^ (t >> 2);
    }
}

constexpr int planes_per_stage(int NB) { return 64 / NB; }   // sources whose masks fit one stage

template <int NB, int D>
__device__ __forceinline__ void wave_tile_planes(const uint8_t *__restrict__ C, int K, int N,
                                                 const uint8_t *__restrict__ S, uint64_t ld_s,
                                                 uint8_t *__restrict__ Y, uint64_t ld_y, uint64_t len, int k0,
                                                 uint64_t p0, bool vec, uint32_t *__restrict__ mk, int lane,
                                                 bool staged)
{
    constexpr int NCP = planes_per_stage(NB);
    static_assert(KW * NCP * NB * 4 <= (int)sizeof(WaveStage), "mask stage exceeds the wave's LDS");
    const uint64_t p = p0 + (uint64_t)lane * (4u * D);
    const uint64_t avail = p < len ? len - p : 0;
    const int kv = min(KW, K - k0);

    uint32_t acc[KW][D];
#pragma unroll
    for (int kk = 0; kk < KW; kk++)
#pragma unroll
        for (int d = 0; d < D; d++)
            acc[kk][d] = 0;

    // the pair of sources in use; the next pair is loaded while it is used
    const uint8_t *src = S + p;
    uint32_t xa[D], xb[D];
    load_lane<D>(src, avail, vec, xa);
    if (N > 1)
        load_lane<D>(src + ld_s, avail, vec, xb);
    else
#pragma unroll
        for (int d = 0; d < D; d++)
            xb[d] = 0;

    for (int g = 0; g < N; g += 2) {
        const int nn = g & (NCP - 1);
        if (nn == 0 && !staged) {
            // masks of rows k0.. and sources g..g+NCP-1: mk[(kk * NCP + j) * NB + b]
            wave_sync();
            const int nc = min(NCP, N - g);
#pragma unroll 4
            for (int it = 0; it < KW * NCP / 64; it++) {
                const int e = lane + 64 * it, kk = e / NCP, j = e % NCP;
                const uint32_t c = (kk < kv && j < nc) ? (uint32_t)gld<uint8_t>(C + (uint64_t)(k0 + kk) * N + g + j) : 0u;
#pragma unroll
                for (int b = 0; b < NB; b++)
                    mk[e * NB + b] = 0u - ((c >> b) & 1u);
            }
            wave_sync();
        }
        uint32_t pa[NB][D], pb[NB][D];
#pragma unroll
        for (int d = 0; d < D; d++) {
            pa[0][d] = xa[d];
            pb[0][d] = xb[d];
#pragma unroll
            for (int b = 1; b < NB; b++) {
                pa[b][d] = times_alpha<NB>(pa[b - 1][d]);
                pb[b][d] = times_alpha<NB>(pb[b - 1][d]);
            }
        }
        // a missing source reads as zero (its masks are zero as well)
        if (g + 2 < N)
            load_lane<D>(src + (uint64_t)(g + 2) * ld_s, avail, vec, xa);
        if (g + 3 < N)
            load_lane<D>(src + (uint64_t)(g + 3) * ld_s, avail, vec, xb);
        else
#pragma unroll
            for (int d = 0; d < D; d++)
                xb[d] = 0;
#pragma unroll
        for (int k8 = 0; k8 < KW; k8 += 8) {
            if (k8 < kv) {
#pragma unroll
                for (int kk = k8; kk < k8 + 8; kk++) {
                    // 2 NB masks: source nn (planes 0..NB-1), then source nn + 1
                    uint32_t m[2 * NB];
                    const uint32_t *mp = mk + (kk * NCP + nn) * NB;
                    if constexpr (NB == 1) {
                        const uint2 v = *reinterpret_cast<const uint2 *>(mp);
                        m[0] = v.x; m[1] = v.y;
                    } else {
#pragma unroll
                        for (int q = 0; q < 2 * NB; q += 4) {
                            const uint4 v = *reinterpret_cast<const uint4 *>(mp + q);
                            m[q] = v.x; m[q + 1] = v.y; m[q + 2] = v.z; m[q + 3] = v.w;
                        }
                    }
#pragma unroll
                    for (int d = 0; d < D; d++) {
                        uint32_t a = acc[kk][d];
#pragma unroll
                        for (int b = 0; b < NB; b++) {
                            a = and_xor(a, pa[b][d], m[b]);
                            a = and_xor(a, pb[b][d], m[NB + b]);
                        }
                        acc[kk][d] = a;
                    }
                }
            }
        }
    }
    if (avail == 0)
        return;
#pragma unroll
    for (int kk = 0; kk < KW; kk++)
        if (kk < kv)
            store_row<D>(Y + (uint64_t)(k0 + kk) * ld_y + p, avail, vec, acc[kk]);
}

// Persistent bit-plane encode over the same wave tiles and queues as the
// table form.
template <int NB>
__global__ __launch_bounds__(256, NB <= 2 ? GF_PLANE_WAVES_PER_SIMD : 2) void k_encode_planes(const DevGen *__restrict__ gens,
                                                                             const DevTile *__restrict__ tiles,
                                                                             const unsigned *__restrict__ runs,
                                                                             const unsigned *__restrict__ bounds,
                                                                             unsigned *counters)
{
    __shared__ WaveStage stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *mk = reinterpret_cast<uint32_t *>(&stage[wave]);
    QueueCursor cursor;
    for (;;) {
        int t = 0;
        if (lane == 0)
            t = queue_next_tile(counters, runs, bounds, cursor);
        t = __builtin_amdgcn_readlane(t, 0);
        if (t < 0)
            break;
        const DevTile tl = tiles[t];
        const DevGen g = gens[tl.gen];
        if (g.status && *g.status != g.need)
            continue;
        const int d = tl.D & 0xFF, strips = (tl.D >> 8) + 1;
        for (int q = 0; q < strips; q++) {
            const uint64_t p0 = tl.p0 + (uint64_t)q * 256u * (uint64_t)d;
            const bool staged = q > 0 && (int)g.N <= planes_per_stage(NB);
            if (d == 4)
                wave_tile_planes<NB, 4>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                                        g.align >= 16, mk, lane, staged);
            else if (d == 2)
                wave_tile_planes<NB, 2>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                                        g.align >= 8, mk, lane, staged);
            else
                wave_tile_planes<NB, 1>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, p0,
                                        g.align >= 4, mk, lane, staged);
        }
    }
    if (lane == 0)
        queue_retire(counters, gridDim.x * WAVES);
}

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
    const int K = (int)g.K, N = (int)g.N;
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

typedef unsigned short gf_u16x2 __attribute__((ext_vector_type(2)));

// The operands of one step: the coefficient bits of the 4 row tiles and the
// source bits of the wave's 2 column tiles.
struct MfOperands {
    gf_v8i a[4];
    gf_v8i b[2];
};

__device__ __forceinline__ void mf_mma(const MfOperands &o, gf_v16f (&acc)[4][2])
{
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        acc[rt][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(o.a[rt], o.b[0], acc[rt][0], 4, 4, 0, 0, 0, 0);
        acc[rt][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(o.a[rt], o.b[1], acc[rt][1], 4, 4, 0, 0, 0, 0);
    }
}

constexpr int kMfRestart = 2048;

// Instruction order for a step's products and the unpacking of the next
// step's operands (whose LDS reads are already issued): two MFMAs while the
// reads are in flight, then the unpacking spread between the remaining six.
__device__ __forceinline__ void mf_step_schedule()
{
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMA
#pragma unroll
    for (int i = 0; i < 6; i++) {
        __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);   // VALU
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
            gf_u16x2 p01, p23;
            uint32_t y[4];
        };
        auto fetch_issue = [&](int zf, int ksf, auto wait_imm) {
            __builtin_amdgcn_s_waitcnt(decltype(wait_imm)::value);
            asm volatile("" ::: "memory");
            const uint16_t *rows = reinterpret_cast<const uint16_t *>(&Sw[wave][zf & (MF_STAGES - 1)][4 * h][0]);
            Raw w;
            w.p01.x = rows[0 * 32 + r];
            w.p01.y = rows[1 * 32 + r];
            w.p23.x = rows[2 * 32 + r];
            w.p23.y = rows[3 * 32 + r];
#pragma unroll
            for (int rt = 0; rt < 4; rt++)
                w.y[rt] = Ybuf[ksf][rt][lane];
            return w;
        };
        auto fetch_unpack = [&](const Raw &w, MfOperands &o) {
            const uint32_t t01 = __builtin_bit_cast(uint32_t, w.p01);   // r0c0 r0c1 r1c0 r1c1
            const uint32_t t23 = __builtin_bit_cast(uint32_t, w.p23);   // r2c0 r2c1 r3c0 r3c1
            o.b[0] = fp4_source(__builtin_amdgcn_perm(t23, t01, 0x06040200u));   // column 2r of rows 0..3
            o.b[1] = fp4_source(__builtin_amdgcn_perm(t23, t01, 0x07050301u));   // column 2r + 1
#pragma unroll
            for (int rt = 0; rt < 4; rt++)
                o.a[rt] = fp4_coef(w.y[rt]);
        };
        // One step: the next operands are read and unpacked while this step's
        // products run (the scheduling fence keeps the reads ahead of them).
        auto step = [&](int zn, int ksn, const MfOperands &cur, MfOperands &nxt, auto wait_imm) {
            const Raw w = fetch_issue(zn, ksn, wait_imm);
            __builtin_amdgcn_sched_barrier(0);
            fetch_unpack(w, nxt);
            mf_mma(cur, acc);
            mf_step_schedule();
        };

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
            for (int kp = 0; kp < npairs; kp++, z += 2) {
                copy_pair();              // pair q + MF_PAIRS_AHEAD, into the slots of pair q - 1
                step(z + 1, 2 * kp + 1, opa, opb, WaitOdd{});
                step(z + 2, kp + 1 == npairs ? 0 : 2 * kp + 2, opb, opa, WaitEven{});   // past the end: a zero slot
            }
            mf_store<true>(g, k0, (uint64_t)strip * MF_STRIP + (uint64_t)wave * 64u + 2u * (uint64_t)r, acc, h,
                           prev, y_even && (uint64_t)(strip + 1) * MF_STRIP <= g.len);
            if ((strip & (kMfRestart - 1)) == kMfRestart - 1) {
                mf_acc_reset(acc);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    prev[i] = 0u;
            }
        }
        // the copies past the last step land before the slots are reused
        __builtin_amdgcn_s_waitcnt(kWaitAll);
        __syncthreads();   // every wave is done with Cl and Ybuf before the next tile
    }
    if (tid == 0)
        queue_retire(counters, gridDim.x);
}

// ------------------------------------------------------------------ invert

// Gauss-Jordan inversion of one N x N matrix (N <= MAXN) in LDS, in place:
// at pivot step j the pivot row is swapped up, its pivot entry replaced by 1
// and the row scaled by the pivot's inverse, then column j is cleared from
// every other row (each such row's column-j entry is first replaced by 0, so
// that after the step it holds the new inverse column).  The row swaps are
// undone at the end as column swaps in reverse order.  Rows are stored with a
// stride of MAXN bytes; a dword holds 4 consecutive entries, and each
// row-times-constant update is one byte-permute product per dword.
// A: the caller's LDS matrix, MAXN rows of MAXN / 4 + 1 dwords; row(r) gives the address
// of the matrix's row r (N bytes, device memory written before this kernel or
// read-only input).
template <int MAXN, class RowOf>
__device__ void invert_rows(uint32_t *A, RowOf row, int N, uint8_t *__restrict__ Cinv, int *rank_out,
                            const uint4 *__restrict__ ptab4, const uint8_t *__restrict__ invg)
{
    constexpr int RW = MAXN / 4;   // dwords of a row
    constexpr int PRW = RW + 1;    // row stride in LDS (odd: a column's bytes spread over the banks)
    __shared__ uint4 T[256][2];
    __shared__ uint8_t IV[256];
    __shared__ uint8_t fcol[MAXN];
    __shared__ int cand[4];
    __shared__ int piv[MAXN];
    __shared__ int src[MAXN];
    uint8_t *Ab = reinterpret_cast<uint8_t *>(A);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NW = (N + 3) >> 2;
    // row updates: thread tid owns column dword cl of rows r0, r0 + RS, ...
    constexpr int RS = 256 / RW;
    const int cl = tid % RW, r0 = tid / RW;

    for (int i = tid; i < 512; i += 256)
        T[i >> 1][i & 1] = ptab4[i];
    IV[tid] = invg[tid];

    auto load_matrix = [&]() {
        for (int i = tid; i < N * RW; i += 256) {
            const int r = i / RW, w = i - r * RW;
            const uint8_t *src = row(r);
            uint32_t v = 0;
            for (int b = 0; b < 4; b++) {
                const int c = 4 * w + b;
                if (c < N)
                    v |= (uint32_t)src[c] << (8 * b);
            }
            A[r * PRW + w] = v;
        }
    };
    // lowest row index >= from with a nonzero entry in column j (>= N if none)
    auto find_pivot = [&](int j, int from) -> int {
        const bool ok = tid < N && tid >= from && Ab[tid * (4 * PRW) + j] != 0;
        const uint64_t m = __ballot(ok);
        if (lane == 0)
            cand[wave] = m ? wave * 64 + __builtin_ctzll(m) : (1 << 30);
        __syncthreads();
        const int pr = min(min(cand[0], cand[1]), min(cand[2], cand[3]));
        return pr;
    };
    auto swap_rows = [&](int a, int b) {
        if (a != b && tid < NW) {
            const uint32_t t = A[a * PRW + tid];
            A[a * PRW + tid] = A[b * PRW + tid];
            A[b * PRW + tid] = t;
        }
    };

    load_matrix();
    __syncthreads();

    bool singular = false;
    for (int j = 0; j < N; j++) {
        const int pr = find_pivot(j, j);
        if (pr >= N) {
            singular = true;
            break;
        }
        swap_rows(pr, j);
        if (tid == 0)
            piv[j] = pr;
        __syncthreads();
        if (tid < NW) {   // wave 0 only: reads below happen before the write
            uint32_t a = A[j * PRW + tid];
            const uint32_t pinv = IV[Ab[j * (4 * PRW) + j]];
            if (tid == (j >> 2))
                a = (a & ~(0xFFu << (8 * (j & 3)))) | (1u << (8 * (j & 3)));
            A[j * PRW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        if (tid < N)
            fcol[tid] = tid == j ? 0 : Ab[tid * (4 * PRW) + j];
        __syncthreads();
        if (cl < NW) {   // thread: column dword cl of rows r0, r0 + RS, ...
            // branch-free: where fcol is 0 the row's byte j is 0 already and the
            // product is 0 (row j itself, whose fcol is 0, keeps its leading 1)
            const uint32_t pj = A[j * PRW + cl];
            const uint32_t keep = cl == (j >> 2) ? ~(0xFFu << (8 * (j & 3))) : 0xFFFFFFFFu;
#pragma unroll 4
            for (int i = r0; i < N; i += RS) {
                const uint32_t f = fcol[i];
                const uint32_t k = i == j ? 0xFFFFFFFFu : keep;
                A[i * PRW + cl] = (A[i * PRW + cl] & k) ^ prod4(T[f][0], T[f][1].x, pj);
            }
        }
        __syncthreads();
    }

    if (!singular) {
        if (tid == 0) {
            for (int c = 0; c < N; c++)
                src[c] = c;
            for (int l = N - 1; l >= 0; l--) {
                const int t = src[l];
                src[l] = src[piv[l]];
                src[piv[l]] = t;
            }
        }
        __syncthreads();
        for (int it = tid; it < N * N; it += 256) {
            const int i = it / N, c = it - i * N;
            Cinv[it] = Ab[i * (4 * PRW) + src[c]];
        }
        if (tid == 0 && rank_out)
            *rank_out = N;
        return;
    }

    // Singular: recompute the exact rank by forward elimination of a fresh copy.
    __syncthreads();
    load_matrix();
    __syncthreads();
    int prow = 0;
    for (int j = 0; j < N && prow < N; j++) {
        const int pr = find_pivot(j, prow);
        if (pr >= N) {
            __syncthreads();
            continue;
        }
        swap_rows(pr, prow);
        __syncthreads();
        if (tid < NW) {
            const uint32_t pinv = IV[Ab[prow * (4 * PRW) + j]];
            const uint32_t a = A[prow * PRW + tid];
            A[prow * PRW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        __syncthreads();
        if (tid < N)
            fcol[tid] = tid > prow ? Ab[tid * (4 * PRW) + j] : 0;
        __syncthreads();
        if (cl < NW) {
            const uint32_t pj = A[prow * PRW + cl];
#pragma unroll 4
            for (int i = r0; i < N; i += RS) {
                const uint32_t f = fcol[i];
                A[i * PRW + cl] ^= prod4(T[f][0], T[f][1].x, pj);
            }
        }
        __syncthreads();
        prow++;
    }
    if (tid == 0 && rank_out)
        *rank_out = prow;
}

// Gauss-Jordan inversion of the row-major N x N matrix at Cg.
template <int MAXN>
__device__ void invert_body(const uint8_t *__restrict__ Cg, int N, uint8_t *__restrict__ Cinv, int *rank_out,
                            const uint4 *__restrict__ ptab4, const uint8_t *__restrict__ invg)
{
    __shared__ uint32_t A[MAXN * (MAXN / 4 + 1)];
    invert_rows<MAXN>(A, [&](int r) { return Cg + (uint64_t)r * N; }, N, Cinv, rank_out, ptab4, invg);
}

template <int MAXN>
__global__ __launch_bounds__(256) void k_invert_one(const uint8_t *__restrict__ C, int N, uint8_t *__restrict__ Cinv,
                                                    int *rank, const uint4 *__restrict__ ptab4,
                                                    const uint8_t *__restrict__ invg)
{
    invert_body<MAXN>(C, N, Cinv, rank, ptab4, invg);
}

template <int MAXN>
__global__ __launch_bounds__(256) void k_invert_batched(const DevSys *__restrict__ sys,
                                                        const uint4 *__restrict__ ptab4,
                                                        const uint8_t *__restrict__ invg)
{
    const DevSys s = sys[blockIdx.x];
    if ((int)s.N > MAXN || (MAXN > 32 && (int)s.N <= MAXN / 2))
        return;   // handled by the launch of another size class
    invert_body<MAXN>(s.C, (int)s.N, s.Cinv, s.rank, ptab4, invg);
}

// ------------------------------------------------------------------ serving

// Progressive decoding of one generation (one workgroup per generation).
// The innovative coefficient vectors received so far are kept in reduced row
// echelon form R.  An arriving vector c is reduced against R in one pass:
// since every row of R is zero in the other rows' pivot columns, subtracting
// c[pivot(r)] * R[r] for all r at once clears every pivot column.  If nothing
// is left the packet carried no new information.  Otherwise c is scaled to a
// leading 1, its pivot column is cleared from the rows of R, and it is stored
// with its raw coefficients and payload.  At rank N the raw coefficient
// matrix is inverted (Gauss-Jordan, as in gf_invert) and the completion step
// is recorded, which releases the payload product S = Csel^-1 * Bsel.
//
// During a step R lives in LDS (the inversion's matrix buffer, free until
// then); packet descriptors are cached 64 at a time and the next packet's
// coefficients are fetched while the current one is reduced, so the loop over
// packets touches device memory only for those prefetches.  The innovative
// packets' raw coefficients and payloads are copied out after the loop.
constexpr int ABSORB_PKC = 64;

__global__ __launch_bounds__(256) void k_absorb(const DevAbsorb *__restrict__ items,
                                                const DevPacket *__restrict__ pkts, const uint4 *__restrict__ ptab4,
                                                const uint8_t *__restrict__ invg)
{
    __shared__ uint32_t Rl[256 * 65];   // row r at Rl + 65 r (odd stride); later the inversion's matrix
    __shared__ uint32_t cw[64];
    __shared__ uint32_t part[4][64];
    __shared__ uint4 T[256][2];
    __shared__ uint8_t IV[256];
    __shared__ uint8_t fcol[256];
    __shared__ int pivc[256];
    __shared__ const uint8_t *row_coef[256];   // raw coefficients of the rows added in this step
    __shared__ const uint8_t *row_pay[256];
    __shared__ DevPacket pkc[ABSORB_PKC];
    __shared__ int cand[4];
    __shared__ int inv_rank;
    const DevAbsorb it = items[blockIdx.x];
    const DevDecSlot &s = it.s;
    const int N = (int)s.N, NW = (N + 3) >> 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint8_t *Rb = reinterpret_cast<const uint8_t *>(Rl);   // row r at byte 260 r

    int rank = s.meta[0];
    if (rank >= N || N > 256)
        return;
    const int rank0 = rank;
    for (int i = tid; i < 512; i += 256)
        T[i >> 1][i & 1] = ptab4[i];
    IV[tid] = invg[tid];
    for (int i = tid; i < rank; i += 256)
        pivc[i] = s.meta[4 + i];
    for (int i = tid; i < rank * NW; i += 256) {
        const int r = i / NW, w = i - r * NW;
        Rl[r * 65 + w] = reinterpret_cast<const uint32_t *>(s.R + (uint64_t)r * s.rs)[w];
    }
    // coefficient dword tid of a packet (lanes tid < NW)
    auto coef_dword = [&](const uint8_t *c) {
        uint32_t v = 0;
        for (int b = 0; b < 4; b++)
            if (4 * tid + b < N)
                v |= (uint32_t)c[4 * tid + b] << (8 * b);
        return v;
    };
    int seen = 0, dropped = 0;
    uint32_t nextv = 0;
    bool have_next = false;

    for (uint32_t q = 0; q < it.npk && rank < N; q++) {
        const int slot = (int)(q % ABSORB_PKC);
        if (slot == 0) {
            __syncthreads();   // every lane is done with the previous descriptors
            if (tid < ABSORB_PKC && q + tid < it.npk)
                pkc[tid] = pkts[it.pk0 + q + tid];
            __syncthreads();
        }
        const DevPacket pk = pkc[slot];
        if (tid < NW)
            cw[tid] = have_next ? nextv : coef_dword(pk.coef);
        // the next packet's coefficients, if its descriptor is cached, land during this one
        have_next = slot + 1 < ABSORB_PKC && q + 1 < it.npk;
        if (have_next && tid < NW)
            nextv = coef_dword(pkc[slot + 1].coef);
        __syncthreads();
        for (int r = tid; r < rank; r += 256) {   // the vector's entry in each row's pivot column
            const int pc = pivc[r];
            fcol[r] = (uint8_t)(cw[pc >> 2] >> (8 * (pc & 3)));
        }
        __syncthreads();
        if (lane < NW) {   // wave w sums rows w, w + 4, ... of column dword `lane`
            uint32_t acc = 0;
#pragma unroll 4
            for (int r = wave; r < rank; r += 4) {   // a zero factor adds a zero product
                const uint32_t f = fcol[r];
                acc ^= prod4(T[f][0], T[f][1].x, Rl[r * 65 + lane]);
            }
            part[wave][lane] = acc;
        }
        __syncthreads();
        if (tid < NW)
            cw[tid] ^= part[0][tid] ^ part[1][tid] ^ part[2][tid] ^ part[3][tid];
        __syncthreads();
        const bool nz = tid < N && ((cw[tid >> 2] >> (8 * (tid & 3))) & 0xFFu) != 0;
        const uint64_t m = __ballot(nz);
        if (lane == 0)
            cand[wave] = m ? wave * 64 + __builtin_ctzll(m) : (1 << 30);
        __syncthreads();
        const int lead = min(min(cand[0], cand[1]), min(cand[2], cand[3]));
        seen++;
        if (lead >= N) {
            dropped++;
            __syncthreads();
            continue;
        }
        if (tid < NW) {   // wave 0 reads the leading entry before any lane rewrites it
            const uint32_t lv = (cw[lead >> 2] >> (8 * (lead & 3))) & 0xFFu;
            const uint32_t iv = IV[lv];
            cw[tid] = prod4(T[iv][0], T[iv][1].x, cw[tid]);
        }
        for (int r = tid; r < rank; r += 256)
            fcol[r] = Rb[r * 260 + lead];
        __syncthreads();
        if (lane < NW) {   // wave w clears the new pivot column from rows w, w + 4, ...
            const uint32_t c = cw[lane];
#pragma unroll 4
            for (int r = wave; r < rank; r += 4) {
                const uint32_t f = fcol[r];
                Rl[r * 65 + lane] ^= prod4(T[f][0], T[f][1].x, c);
            }
        }
        if (tid < NW)
            Rl[rank * 65 + tid] = cw[tid];
        if (tid == 0) {
            pivc[rank] = lead;
            row_coef[rank] = pk.coef;
            row_pay[rank] = pk.payload;
        }
        rank++;
        __syncthreads();
    }
    // R back to device memory; the new rows' raw coefficients and payloads
    for (int i = tid; i < rank * NW; i += 256) {
        const int r = i / NW, w = i - r * NW;
        reinterpret_cast<uint32_t *>(s.R + (uint64_t)r * s.rs)[w] = Rl[r * 65 + w];
    }
    for (int rr = rank0; rr < rank; rr++) {
        const uint8_t *pc = row_coef[rr];
        for (int b = tid; b < N; b += 256)
            s.Csel[(uint64_t)rr * N + b] = pc[b];
        const uint8_t *src = row_pay[rr];
        uint8_t *dst = s.Bsel + (uint64_t)rr * s.ld;
        if (((((uintptr_t)dst) | ((uintptr_t)src)) & 3u) == 0) {
            const uint64_t words = s.len >> 2;
            for (uint64_t w = tid; w < words; w += 256)
                reinterpret_cast<uint32_t *>(dst)[w] = reinterpret_cast<const uint32_t *>(src)[w];
            for (uint64_t b = (words << 2) + tid; b < s.len; b += 256)
                dst[b] = src[b];
        } else {
            for (uint64_t b = tid; b < s.len; b += 256)
                dst[b] = src[b];
        }
    }
    for (int i = tid; i < rank; i += 256)
        s.meta[4 + i] = pivc[i];
    if (tid == 0) {
        s.meta[0] = rank;
        s.meta[2] += seen;
        s.meta[3] += dropped;
    }
    if (rank == N) {
        __syncthreads();   // Rl is free: the inversion reads the raw rows from their sources
        invert_rows<256>(Rl,
                         [&](int r) {
                             return r < rank0 ? s.Csel + (uint64_t)r * N : row_coef[r];
                         },
                         N, s.Cinv, &inv_rank, ptab4, invg);
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            s.meta[1] = it.step;
        }
    }
}

__global__ void k_meta_init(int *const *__restrict__ metas, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int *m = metas[i];
        m[0] = 0;
        m[1] = -1;
        m[2] = 0;
        m[3] = 0;
    }
}

__global__ void k_status_gather(int *const *__restrict__ metas, int n, int4 *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int *m = metas[i];
        out[i] = make_int4(m[0], m[1], m[2], m[3]);
    }
}

}  // namespace

// ----------------------------------------------------------------- launchers

hipError_t launch_region(int mode, uint8_t *y, const uint8_t *x, uint64_t len, const uint32_t *t, hipStream_t s)
{
    if (len == 0)
        return hipSuccess;
    const int vec = ((((uintptr_t)y) ^ ((uintptr_t)x)) & 15u) == 0;
    uint64_t blocks = (len / 16 + 511) / 512;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 256 * 16)
        blocks = 256 * 16;
    if (mode == 0)
        hipLaunchKernelGGL(k_region<0>, dim3((unsigned)blocks), dim3(256), 0, s, y, x, len, t[0], t[1], t[2], t[3],
                           t[4], vec);
    else
        hipLaunchKernelGGL(k_region<1>, dim3((unsigned)blocks), dim3(256), 0, s, y, x, len, t[0], t[1], t[2], t[3],
                           t[4], vec);
    return hipGetLastError();
}

hipError_t launch_region_batched(const void *d_regions, int count, uint64_t max_len, const uint32_t *ptab_field,
                                 int q, hipStream_t s)
{
    if (count <= 0 || max_len == 0)
        return hipSuccess;
    const uint64_t gx = (max_len + REGION_CHUNK - 1) / REGION_CHUNK;
    // grid.y is limited to 65535: split the region list into slices
    for (int base = 0; base < count; base += 65535) {
        const int n = min(65535, count - base);
        hipLaunchKernelGGL(k_region_batched, dim3((unsigned)gx, (unsigned)n), dim3(256), 0, s,
                           reinterpret_cast<const RegionDesc *>(d_regions) + base,
                           reinterpret_cast<const uint4 *>(ptab_field), q);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_encode(int D, int nsplit, const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s,
                         uint8_t *Y, uint64_t ld_y, uint64_t len, const uint32_t *ptab_field, const int *status,
                         int need, bool aligned, hipStream_t s)
{
    if (K <= 0 || len == 0)
        return hipSuccess;
    if (nsplit < 1 || nsplit > N)
        nsplit = 1;
    const uint64_t strip = 256u * (uint64_t)D;
    const uint64_t nstrips = (len + strip - 1) / strip;
    const uint64_t ntiles = nstrips * (uint64_t)nsplit * (uint64_t)((K + KW - 1) / KW);
    if (ntiles > 0xFFFFFFFFull / 2)
        return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((ntiles + WAVES - 1) / WAVES);
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    const int vec = aligned ? 1 : 0;
    if (nsplit > 1) {
        const uint64_t words = (len / 4) * (uint64_t)K;
        if (words > 0) {
            const unsigned zb = (unsigned)std::min<uint64_t>((words + 255) / 256, 4096);
            hipLaunchKernelGGL(k_zero_rows, dim3(zb), dim3(256), 0, s, Y, ld_y, len, K, status, need);
        }
        if (len & 3) {
            const unsigned tb = (unsigned)((K * (int)(len & 3) + 255) / 256);
            hipLaunchKernelGGL(k_encode_tail, dim3(tb), dim3(256), 0, s, C, K, N, S, ld_s, Y, ld_y, len, pt, status,
                               need);
        }
    }
#define GF_DIRECT(DD)                                                                                            \
    hipLaunchKernelGGL(k_encode_direct<DD>, dim3(blocks), dim3(256), 0, s, C, K, N, S, ld_s, Y, ld_y, len, pt,   \
                       status, need, vec, (uint32_t)nstrips, (uint32_t)nsplit, (uint32_t)ntiles)
    if (D == 4)
        GF_DIRECT(4);
    else if (D == 2)
        GF_DIRECT(2);
    else if (D == 1)
        GF_DIRECT(1);
    else
        return hipErrorInvalidValue;
#undef GF_DIRECT
    return hipGetLastError();
}

hipError_t launch_encode_persistent(const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                    const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                    const uint32_t *ptab_field, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_encode_waves, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters,
                       reinterpret_cast<const uint4 *>(ptab_field));
    return hipGetLastError();
}

hipError_t launch_encode_planes(int field, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (field == 1)
        hipLaunchKernelGGL(k_encode_planes<1>, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters);
    else if (field == 2)
        hipLaunchKernelGGL(k_encode_planes<2>, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters);
    else if (field == 4)
        hipLaunchKernelGGL(k_encode_planes<4>, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int encode_planes_blocks_per_cu(int field)
{
    const void *k = field == 1   ? reinterpret_cast<const void *>(&k_encode_planes<1>)
                    : field == 2 ? reinterpret_cast<const void *>(&k_encode_planes<2>)
                                 : reinterpret_cast<const void *>(&k_encode_planes<4>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess || nb < 1)
        return 1;
    return nb;
}

int encode_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_encode_waves), 256, 0) !=
            hipSuccess ||
        nb < 1)
        return 1;
    return nb;
}

hipError_t launch_invert(const DevSys *sys, int count, const uint8_t *C, int N, uint8_t *Cinv, int *rank,
                         const uint32_t *ptab_field, const uint8_t *inv_field, hipStream_t s)
{
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    if (sys == nullptr) {
        if (N <= 32)
            hipLaunchKernelGGL(k_invert_one<32>, dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        else if (N <= 64)
            hipLaunchKernelGGL(k_invert_one<64>, dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        else if (N <= 128)
            hipLaunchKernelGGL(k_invert_one<128>, dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        else
            hipLaunchKernelGGL(k_invert_one<256>, dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        return hipGetLastError();
    }
    if (count <= 0)
        return hipSuccess;
    // One launch per size class; each block skips systems of other classes.
    hipLaunchKernelGGL(k_invert_batched<32>, dim3(count), dim3(256), 0, s, sys, pt, inv_field);
    hipLaunchKernelGGL(k_invert_batched<64>, dim3(count), dim3(256), 0, s, sys, pt, inv_field);
    hipLaunchKernelGGL(k_invert_batched<128>, dim3(count), dim3(256), 0, s, sys, pt, inv_field);
    hipLaunchKernelGGL(k_invert_batched<256>, dim3(count), dim3(256), 0, s, sys, pt, inv_field);
    return hipGetLastError();
}

hipError_t launch_absorb(const DevAbsorb *items, int n, const DevPacket *pkts, const uint32_t *ptab_field,
                         const uint8_t *inv_field, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_absorb, dim3(n), dim3(256), 0, s, items, pkts, reinterpret_cast<const uint4 *>(ptab_field),
                       inv_field);
    return hipGetLastError();
}

hipError_t launch_meta_init(int *const *metas, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_meta_init, dim3((n + 255) / 256), dim3(256), 0, s, metas, n);
    return hipGetLastError();
}

hipError_t launch_status_gather(int *const *metas, int n, int4 *out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_status_gather, dim3((n + 255) / 256), dim3(256), 0, s, metas, n, out);
    return hipGetLastError();
}

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
    int nb = 0;
    const void *k = aligned4 ? reinterpret_cast<const void *>(&k_encode_mfma_dma)
                              : reinterpret_cast<const void *>(&k_encode_mfma);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) !=
            hipSuccess ||
        nb < 1)
        return 1;
    return nb;
}

}  // namespace gfnc
