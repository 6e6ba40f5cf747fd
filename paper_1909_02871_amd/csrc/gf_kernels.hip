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
#include "gf_queue.h"

namespace gfnc {

namespace {

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

// The same for data touched once (streamed sources and outputs): marked
// non-temporal, so they pass through the caches without displacing what is
// reused.
template <class T>
__device__ __forceinline__ T gld_nt(const void *p)
{
    return __builtin_nontemporal_load(
        reinterpret_cast<const __attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p)));
}

template <class T>
__device__ __forceinline__ void gst_nt(void *p, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<__attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p)));
}

// Bytes [q, q + 4D) of a row, as D dwords: q is the row's byte `off`, and
// `avail` bytes of the row are left from there.  vec: the row starts 16-byte
// aligned and off is a multiple of 4D.  Then the block is read with one
// vector load, unconditionally, also when the row ends inside it: an aligned
// block of at most 16 bytes lies inside the 4 KiB page of its first byte, so
// the read stays in mapped memory; a block wholly past the end reads the
// row's first block instead.  Either way the bytes past the row's end hold
// other data.  Every caller multiplies byte positions independently and stores
// only the first `avail` bytes of its results, so they never reach an output.
// (Masking them here, or a branch around the load, would use the loaded value
// at once, and a wave that uses a load waits for every load it has in flight,
// which would empty the callers' software pipelines.)  Rows that are not
// aligned go byte by byte, zero past the end.
template <int D, bool NT = false>
__device__ __forceinline__ void load_row(const uint8_t *q, uint64_t off, uint64_t avail, bool vec, uint32_t (&x)[D])
{
    if (vec) {
        const uint8_t *a = avail > 0 ? q : q - off;
        if constexpr (D == 4 && NT) {
            const gf_u32x4 t = gld_nt<gf_u32x4>(a);
            x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
        } else if constexpr (D == 4) {
            const gf_u32x4 t = gld<gf_u32x4>(a);
            x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
        } else if constexpr (D == 2) {
            const gf_u32x2 t = gld<gf_u32x2>(a);
            x[0] = t.x; x[1] = t.y;
        } else {
            x[0] = gld<uint32_t>(a);
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; d++)
            x[d] = 0;
#pragma unroll
        for (int b = 0; b < 4 * D; b++)
            if ((uint64_t)b < avail)
                x[b >> 2] |= (uint32_t)gld<uint8_t>(q + b) << (8 * (b & 3));
    }
}

template <int D, bool NT = false>
__device__ __forceinline__ void store_row(uint8_t *p, uint64_t avail, bool vec, const uint32_t (&x)[D])
{
    if (vec && avail >= 4u * D) {
        if constexpr (D == 4 && NT) {
            gst_nt<gf_u32x4>(p, gf_u32x4{x[0], x[1], x[2], x[3]});
        } else if constexpr (D == 4) {
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

// One 16-byte piece of a batched region madd: bytes [p, p + 16) of region d
// (p < d.len, a multiple of 16).  When x and y are 16-byte aligned, both
// pieces are read with one vector load each, also the region's last, partial
// piece: an aligned 16-byte block lies inside the 4 KiB page of its first
// byte, so reading it whole stays in mapped memory; only the bytes before
// d.len are written back.  Unaligned regions load every byte first and then
// store, so the wave waits for its loads once.
// y[p .. p + 16) ^= c x[p .. p + 16) from loaded 16-byte pieces of an
// aligned region, stored whole or (the region's last piece) by words and bytes
// up to its end; nothing is stored for a piece at or past the end.
__device__ __forceinline__ void region_store(uint8_t *y, uint64_t p, uint64_t len, const uint4 ta, uint32_t tb,
                                             const gf_u32x4 &xv, gf_u32x4 v)
{
    v.x ^= prod4(ta, tb, xv.x);
    v.y ^= prod4(ta, tb, xv.y);
    v.z ^= prod4(ta, tb, xv.z);
    v.w ^= prod4(ta, tb, xv.w);
    if (p + 16 <= len) {
        gst_nt<gf_u32x4>(y + p, v);
    } else if (p < len) {
        const int n = (int)(len - p);   // 1 .. 15 bytes left
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (4 * k + 4 <= n)
                gst<uint32_t>(y + p + 4 * k, w[k]);
#pragma unroll
        for (int b = 0; b < 16; b++)
            if (b >= (n & ~3) && b < n)
                gst<uint8_t>(y + p + b, (uint8_t)(w[b >> 2] >> (8 * (b & 3))));
    }
}

__device__ __forceinline__ void region_piece(const RegionDesc &d, uint64_t p, const uint4 ta, uint32_t tb)
{
    if ((((uintptr_t)d.y | (uintptr_t)d.x) & 15u) == 0) {
        const gf_u32x4 a = gld_nt<gf_u32x4>(d.x + p);
        const gf_u32x4 yv = gld_nt<gf_u32x4>(d.y + p);
        region_store(d.y, p, d.len, ta, tb, a, yv);
    } else {
        const int n = (int)(min(d.len, p + 16) - p);
        uint32_t xb[16], yb[16];
#pragma unroll
        for (int b = 0; b < 16; b++) {
            const uint64_t o = p + (uint64_t)(b < n ? b : n - 1);   // inside the region
            xb[b] = gld<uint8_t>(d.x + o);
            yb[b] = gld<uint8_t>(d.y + o);
        }
#pragma unroll
        for (int b = 0; b < 16; b++)
            if (b < n)
                gst<uint8_t>(d.y + p + b, (uint8_t)(yb[b] ^ (prod4(ta, tb, xb[b]) & 0xFFu)));
    }
}

// Batched madd of regions shorter than 4 KiB: one wave per region at a time
// (regions dealt to the waves round robin; the launcher starts a wave for
// every region, so each takes one), lane l taking the 16-byte pieces
// l, l + 64, ..., M per lane (M = 1024-byte rounds of the longest region).
// Descriptors and the coefficient's tables are wave-uniform scalar loads, the
// next region's read while the current one's pieces are in flight.  For
// 16-byte aligned regions the wave issues the loads of all its pieces of x
// and y back to back (a piece past the region's end re-reads its first
// piece), waits once, and stores the pieces inside the region; others go
// piece by piece.
constexpr int REGION_WAVES = 4;   // waves per workgroup of the region kernels

__device__ __forceinline__ bool region_live(const RegionDesc &d, int q)
{
    return d.c != 0 && d.c < (uint32_t)q && d.len != 0;
}

template <int M>
__global__ __launch_bounds__(256) void k_region_waves(const RegionDesc *__restrict__ regs,
                                                      const uint4 *__restrict__ ptab4, int q, int count)
{
    const int lane = threadIdx.x & 63;
    const int w0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * REGION_WAVES) + (int)(threadIdx.x >> 6));
    const int nw = (int)(gridDim.x * REGION_WAVES);
    if (w0 >= count)
        return;
    RegionDesc d = regs[w0];
    uint4 ta = ptab4[d.c < 256 ? d.c * 2 : 0];
    uint32_t tb = ptab4[d.c < 256 ? d.c * 2 + 1 : 1].x;
    for (int r = w0; r < count; r += nw) {
        const int rn = r + nw;
        const RegionDesc dn = regs[min(rn, count - 1)];   // one scalar load, unconditional
        const bool live = region_live(d, q);
        if (live && ((((uintptr_t)d.y | (uintptr_t)d.x)) & 15u) == 0) {
            gf_u32x4 xv[M], yv[M];
#pragma unroll
            for (int m = 0; m < M; m++) {
                const uint64_t pc = (uint64_t)(lane + 64 * m) * 16u;
                const uint64_t p = pc < d.len ? pc : 0;   // in the region, so in mapped memory
                xv[m] = gld_nt<gf_u32x4>(d.x + p);
                yv[m] = gld_nt<gf_u32x4>(d.y + p);
            }
#pragma unroll
            for (int m = 0; m < M; m++) {
                // every loaded register is read here, also for pieces past the
                // end, so no load is left in flight for the next region's loads
                // to wait on (they would wait for this region's stores too)
                asm volatile("" ::"v"(xv[m].x), "v"(xv[m].y), "v"(xv[m].z), "v"(xv[m].w));
                asm volatile("" ::"v"(yv[m].x), "v"(yv[m].y), "v"(yv[m].z), "v"(yv[m].w));
                region_store(d.y, (uint64_t)(lane + 64 * m) * 16u, d.len, ta, tb, xv[m], yv[m]);
            }
        } else if (live) {
#pragma unroll
            for (int m = 0; m < M; m++) {
                const uint64_t p = (uint64_t)(lane + 64 * m) * 16u;
                if (p < d.len)
                    region_piece(d, p, ta, tb);
            }
        }
        if (rn < count) {   // the next region's tables, read while its data are fetched
            ta = ptab4[dn.c < 256 ? dn.c * 2 : 0];
            tb = ptab4[dn.c < 256 ? dn.c * 2 + 1 : 1].x;
        }
        d = dn;
    }
}

// Regions of 4 KiB and more: block (bx, r) handles bytes [bx*REGION_CHUNK, ...)
// of region r, with the region's descriptor and tables loaded once per block.
// (Two or four pieces per thread, loads first, measured slower at 9000 B and
// 64 KiB.)
constexpr int REGION_CHUNK = 256 * 16;   // bytes per block per region

__global__ __launch_bounds__(256) void k_region_chunks(const RegionDesc *__restrict__ regs,
                                                       const uint4 *__restrict__ ptab4, int q)
{
    const RegionDesc d = regs[blockIdx.y];
    const uint64_t start = (uint64_t)blockIdx.x * REGION_CHUNK;
    if (d.c == 0 || d.c >= (uint32_t)q || start >= d.len)
        return;
    const uint4 ta = ptab4[d.c * 2];
    const uint32_t tb = ptab4[d.c * 2 + 1].x;
    const uint64_t p = start + threadIdx.x * 16u;
    if (p < d.len)
        region_piece(d, p, ta, tb);
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
    load_row<D>(src + (uint64_t)nb * ld_s, p, avail, vec, xa);
    if (nb + 1 < ne)
        load_row<D>(src + (uint64_t)(nb + 1) * ld_s, p, avail, vec, xb);
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
            load_row<D>(src + (uint64_t)(g + 2) * ld_s, p, avail, vec, xa);
        if (g + 3 < ne)
            load_row<D>(src + (uint64_t)(g + 3) * ld_s, p, avail, vec, xb);
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

// ----------------------------------------------------- small generations
//
// Batches whose generations all have K <= 8 coded rows and N <= 8 sources do
// little arithmetic per byte (K byte-madds), so they are bound by memory
// latency and bandwidth, not by the lookups.  A wave here takes a tile of up
// to STREAM_STRIPS strips of 1 KiB (16 bytes per lane) of one generation,
// stages the generation's K x N product tables in its LDS once, and streams
// the strips in bursts of B: the loads of B strips go out back to back, the
// wave waits for them once, multiplies the B strips and stores them.  (On
// this chip loads and stores share one completion counter that the compiler
// must treat as unordered once both are in flight, so a wave cannot keep a
// load in flight across the use of an earlier one while its stores drain;
// what it can do is issue many loads before its first use.)  SK (the batch's
// largest K or N, rounded up to 1, 2, 4 or 8) sizes the registers, and B
// shrinks as SK grows, so every burst reads about 8 KiB; the small register
// budget lets 8 waves share each SIMD, whose bursts overlap.

template <int SK>
struct SmallStage {
    uint4 t[SK][SK][2];   // [coded row][source][tables]
};

// The source rows x 16 bytes of one strip per lane; rows are 16-byte
// aligned.  Rows past N re-read row N - 1 (their tables are zero), so every
// load is unconditional: a wave whose loads all feed the next products never
// has a stale load in flight when it reuses the registers.
template <int SK>
__device__ __forceinline__ void small_load(const uint8_t *S, uint64_t ld_s, int N, uint64_t p, uint64_t len,
                                           uint32_t (&x)[SK][4])
{
    const uint64_t avail = p < len ? len - p : 0;
#pragma unroll
    for (int i = 0; i < SK; i++)
        load_row<4, true>(S + (uint64_t)min(i, N - 1) * ld_s + p, p, avail, true, x[i]);
}

// All K coded rows of one strip: the sources go two at a time (their byte
// splits computed once), each pair multiplied into every row's accumulators.
template <int SK>
__device__ __forceinline__ void small_strip(const SmallStage<SK> &st, int K, int N, uint8_t *Y, uint64_t ld_y,
                                            uint64_t p, uint64_t len, bool vec, const uint32_t (&x)[SK][4],
                                            bool store = true)
{
    const uint64_t avail = p < len && store ? len - p : 0;
    uint32_t acc[SK][4];
#pragma unroll
    for (int k = 0; k < SK; k++)
#pragma unroll
        for (int d = 0; d < 4; d++)
            acc[k][d] = 0;
#pragma unroll
    for (int i = 0; i < SK; i += 2) {
        if (i >= N)
            break;
        const bool two = i + 1 < SK;
        Sel sa[4], sb[4];
#pragma unroll
        for (int d = 0; d < 4; d++) {
            sa[d] = split(x[i][d]);
            sb[d] = split(two ? x[i + 1 < SK ? i + 1 : i][d] : 0u);   // zero past N, with zero tables
        }
#pragma unroll
        for (int k = 0; k < SK; k++) {
            if (k >= K)
                break;
            const uint4 a = st.t[k][i][0];
            const uint32_t b = st.t[k][i][1].x;
            const uint4 a2 = two ? st.t[k][i + 1 < SK ? i + 1 : i][0] : uint4{0, 0, 0, 0};
            const uint32_t b2 = two ? st.t[k][i + 1 < SK ? i + 1 : i][1].x : 0u;
#pragma unroll
            for (int d = 0; d < 4; d++) {
                const uint32_t p0 = __builtin_amdgcn_perm(a.y, a.x, sa[d].a);
                const uint32_t p1 = __builtin_amdgcn_perm(a.w, a.z, sa[d].b);
                const uint32_t p2 = __builtin_amdgcn_perm(b, b, sa[d].c);
                if (two) {
                    const uint32_t q0 = __builtin_amdgcn_perm(a2.y, a2.x, sb[d].a);
                    const uint32_t q1 = __builtin_amdgcn_perm(a2.w, a2.z, sb[d].b);
                    const uint32_t q2 = __builtin_amdgcn_perm(b2, b2, sb[d].c);
                    acc[k][d] = xor3(xor3(xor3(acc[k][d], p0, p1), p2, q0), q1, q2);
                } else {
                    acc[k][d] = xor3(acc[k][d], p0, p1) ^ p2;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < SK; k++)
        if (k < K)
            store_row<4, true>(Y + (uint64_t)k * ld_y + p, avail, vec, acc[k]);
}

// queue_next_tile for a whole wave, every lane calling with the same cursor: lane 0
// makes the claims, every other load is from a wave-uniform address, and the
// result is wave-uniform.  While the current run lasts no memory is touched,
// so a wave that claims its next tile early does not wait for the loads and
// stores it has in flight.
__device__ __forceinline__ int queue_next_tile_wave(unsigned *counters, const unsigned *__restrict__ runs,
                                                    const unsigned *__restrict__ bounds, QueueCursor &c, int lane)
{
    const int home = (int)(blockIdx.x % MF_QUEUES);
    while (c.next == c.end) {
        if (c.q >= MF_QUEUES)
            return -1;
        const int qi = (home + c.q) % MF_QUEUES;
        const unsigned lo = bounds[qi], hi = bounds[qi + 1];
        unsigned t = ~0u;
        if (lo < hi) {
            unsigned v = 0;
            if (lane == 0)
                v = atomicAdd(&counters[MF_CTR_STRIDE * qi], 1u);
            t = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
        }
        if (lo < hi && t < hi - lo) {
            const unsigned r = lo + t;
            c.next = runs ? runs[r] : r;
            c.end = runs ? runs[r + 1] : r + 1;
        } else {
            c.q++;
        }
    }
    return (int)c.next++;
}

// A tile descriptor made wave-uniform (each field taken from lane 0), so that
// loops and branches over its strips stay scalar.
__device__ __forceinline__ DevTile uniform_tile(const DevTile &v)
{
    DevTile u;
    u.gen = __builtin_amdgcn_readfirstlane(v.gen);
    u.k0 = (uint16_t)__builtin_amdgcn_readfirstlane((uint32_t)v.k0);
    u.D = (uint16_t)__builtin_amdgcn_readfirstlane((uint32_t)v.D);
    u.p0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v.p0 >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v.p0);
    return u;
}

// Tile t, read as one 16-byte word from a wave-uniform address.
__device__ __forceinline__ DevTile read_tile(const DevTile *__restrict__ tiles, int t)
{
    const uint4 w = reinterpret_cast<const uint4 *>(tiles)[t];
    DevTile v;
    v.gen = w.x;
    v.k0 = (uint16_t)(w.y & 0xFFFFu);
    v.D = (uint16_t)(w.y >> 16);
    v.p0 = ((uint64_t)w.w << 32) | w.z;
    return uniform_tile(v);
}

// Marks every loaded dword of a strip as read, on every path through the
// products (rows past N skip them): the compiler then knows no load into these
// registers is still in flight when the next burst reuses them, and does not
// make that burst wait for the stores in flight as well.
template <int SK>
__device__ __forceinline__ void hold(const uint32_t (&x)[SK][4])
{
#pragma unroll
    for (int i = 0; i < SK; i++)
#pragma unroll
        for (int d = 0; d < 4; d++)
            asm volatile("" ::"v"(x[i][d]));
}

// One burst of R strips from strip s0: the R strips' loads go out back to
// back, then (first burst of a tile) the coefficients' product tables are
// looked up in the block's LDS copy of the field table and staged, then the
// strips are multiplied and stored in order.
template <int SK, int R>
__device__ __forceinline__ void stream_burst(const DevGen &g, int K, int N, uint64_t p0, int s0, SmallStage<SK> &st,
                                             const uint4 *field_tab, int lane, bool first, uint32_t c, bool has_c)
{
    uint32_t x[R][SK][4];
#pragma unroll
    for (int u = 0; u < R; u++)
        small_load<SK>(g.S, g.ld_s, N, p0 + (uint64_t)(s0 + u) * 1024u, g.len, x[u]);
    if (first) {
        const int k = lane / SK, i = lane % SK;
        const uint32_t cv = has_c ? c : 0u;
        wave_sync();
        if (lane < SK * SK) {   // one (row, source) pair per lane; zero tables past K or N
            st.t[k][i][0] = field_tab[cv * 2];
            st.t[k][i][1] = field_tab[cv * 2 + 1];
        }
        wave_sync();
    }
#pragma unroll
    for (int u = 0; u < R; u++) {
        small_strip<SK>(st, K, N, g.Y, g.ld_y, p0 + (uint64_t)(s0 + u) * 1024u, g.len, true, x[u]);
        hold<SK>(x[u]);
    }
}

// The strips s0 .. s0 + rem - 1 (rem < B) as one burst of exactly that many.
template <int SK, int R>
__device__ __forceinline__ void stream_rest(const DevGen &g, int K, int N, uint64_t p0, int s0, int rem,
                                            SmallStage<SK> &st, const uint4 *field_tab, int lane, bool first,
                                            uint32_t c, bool has_c)
{
    if constexpr (R >= 1) {
        if (rem == R)
            stream_burst<SK, R>(g, K, N, p0, s0, st, field_tab, lane, first, c, has_c);
        else
            stream_rest<SK, R - 1>(g, K, N, p0, s0, rem, st, field_tab, lane, first, c, has_c);
    }
}

// One tile of the streaming form.  The claim of the wave's next tile comes
// first (it touches memory only when the wave's run of tiles is used up),
// then the K x N coefficient bytes and the first burst; the next tile's
// descriptor is read while the burst is in flight.  Bursts are B strips, the
// last one exactly the strips that are left.  Returns the next tile (or -1)
// with its descriptor in `next`.
template <int SK, int B>
__device__ __forceinline__ int stream_tile(const DevGen &g, const DevTile &tl, SmallStage<SK> &st,
                                           const uint4 *field_tab, int lane, const DevTile *__restrict__ tiles,
                                           const unsigned *__restrict__ runs, const unsigned *__restrict__ bounds,
                                           unsigned *counters, QueueCursor &cursor, DevTile &next)
{
    const int tn = queue_next_tile_wave(counters, runs, bounds, cursor, lane);
    const int K = (int)g.K, N = (int)g.N, n = (tl.D >> 8) + 1;   // strips of the tile
    const uint64_t p0 = tl.p0 + (uint64_t)lane * 16u;
    const int k = lane / SK, i = lane % SK;
    const bool has_c = lane < SK * SK && k < K && i < N;
    // every lane reads a coefficient byte (lanes past K x N read C[0])
    const uint32_t c = gld<uint8_t>(g.C + (has_c ? (uint64_t)k * N + i : 0));
    if (tn >= 0)
        next = read_tile(tiles, tn);
    int s0 = 0;
    bool first = true;
    for (; s0 + B <= n; s0 += B) {
        stream_burst<SK, B>(g, K, N, p0, s0, st, field_tab, lane, first, c, has_c);
        first = false;
    }
    if (s0 < n)
        stream_rest<SK, B - 1>(g, K, N, p0, s0, n - s0, st, field_tab, lane, first, c, has_c);
    return tn;
}

// Waves per SIMD each instance is built for: every burst reads about 8 KiB,
// and the more waves share a SIMD, the more bursts are in flight.
constexpr int stream_waves(int sk) { return sk <= 1 ? 6 : sk <= 2 ? 4 : sk <= 4 ? 3 : 2; }

template <int SK, int B>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stream_waves(SK)))) void k_encode_stream(const DevGen *__restrict__ gens,
                                                       const DevTile *__restrict__ tiles,
                                                       const unsigned *__restrict__ runs,
                                                       const unsigned *__restrict__ bounds, unsigned *counters,
                                                       const uint4 *__restrict__ ptab4)
{
    __shared__ uint4 field_tab[256 * 2];
    __shared__ SmallStage<SK> stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < 256 * 2; e += 256)
        field_tab[e] = ptab4[e];
    __syncthreads();
    QueueCursor cursor;
    int t = queue_next_tile_wave(counters, runs, bounds, cursor, lane);
    DevTile tl{};
    if (t >= 0)
        tl = read_tile(tiles, t);
    while (t >= 0) {
        const DevGen g = gens[tl.gen];
        DevTile next{};
        int tn;
        const bool run = !g.status || __builtin_amdgcn_readfirstlane((uint32_t)*g.status) == (uint32_t)g.need;
        if (!run) {   // a generation not to run: claim the next tile
            tn = queue_next_tile_wave(counters, runs, bounds, cursor, lane);
            if (tn >= 0)
                next = read_tile(tiles, tn);
        } else {
            tn = stream_tile<SK, B>(g, tl, stage[wave], field_tab, lane, tiles, runs, bounds, counters, cursor,
                                    next);
        }
        // the loop's control stays scalar: the next tile's index and descriptor as lane 0 has them
        t = __builtin_amdgcn_readfirstlane(tn);
        tl = uniform_tile(next);
    }
    if (lane == 0)
        queue_retire(counters, gridDim.x * WAVES);
}

// The same small generations dealt out by the hardware instead of queues:
// wave w of workgroup b takes tile 4b + w, a run of at most B strips of one
// generation (its strips split into runs of equal length), as one burst, and
// the launch has a workgroup per four tiles.  No wave outlives its burst, so
// no loads wait behind a previous burst's stores; the coefficients' tables
// come straight from the field table in global memory (a few L2 hits per
// wave) instead of a per-workgroup LDS copy.
template <int SK, int B>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stream_waves(SK)))) void k_encode_chunks(
    const DevGen *__restrict__ gens, const DevTile *__restrict__ tiles, int ntiles, const uint4 *__restrict__ ptab4)
{
    __shared__ SmallStage<SK> stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WAVES + wave);
    if (t >= ntiles)
        return;
    const DevTile tl = read_tile(tiles, t);
    const DevGen g = gens[tl.gen];
    if (g.status && __builtin_amdgcn_readfirstlane((uint32_t)*g.status) != (uint32_t)g.need)
        return;
    const int K = (int)g.K, N = (int)g.N, n = (tl.D >> 8) + 1;
    const int k = lane / SK, i = lane % SK;
    const bool has_c = lane < SK * SK && k < K && i < N;
    const uint32_t c = gld<uint8_t>(g.C + (has_c ? (uint64_t)k * N + i : 0));
    stream_rest<SK, B>(g, K, N, tl.p0 + (uint64_t)lane * 16u, 0, n, stage[wave], ptab4, lane, true, c, has_c);
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

// Persistent encode over the work queues; every wave claims tiles on its own.
template <bool DIRECT = false>
__global__ __launch_bounds__(256, GF_ENC_WAVES_PER_SIMD) void k_encode_waves(const DevGen *__restrict__ gens,
                                                      const DevTile *__restrict__ tiles,
                                                      const unsigned *__restrict__ runs,
                                                      const unsigned *__restrict__ bounds, unsigned *counters,
                                                      const uint4 *__restrict__ ptab4, int ntiles)
{
    __shared__ WaveStage stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    QueueCursor cursor;
    for (int pass = 0;; pass++) {
        int t = 0;
        if constexpr (DIRECT) {   // not persistent: wave w of workgroup b takes tile 4b + w only
            t = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WAVES + wave);
            if (pass > 0 || t >= ntiles)
                break;
        } else {
            if (lane == 0)
                t = queue_next_tile(counters, runs, bounds, cursor);
            t = __builtin_amdgcn_readlane(t, 0);
            if (t < 0)
                break;
        }
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
    if (!DIRECT && lane == 0)
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
    load_row<D>(src, p, avail, vec, xa);
    if (N > 1)
        load_row<D>(src + ld_s, p, avail, vec, xb);
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
            load_row<D>(src + (uint64_t)(g + 2) * ld_s, p, avail, vec, xa);
        if (g + 3 < N)
            load_row<D>(src + (uint64_t)(g + 3) * ld_s, p, avail, vec, xb);
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
// table form.  DIRECT: not persistent; wave w of workgroup b takes tile 4b + w
// of the list and nothing else (a workgroup per four tiles).
template <int NB, bool DIRECT = false>
__global__ __launch_bounds__(256, NB <= 2 ? GF_PLANE_WAVES_PER_SIMD : 2) void k_encode_planes(const DevGen *__restrict__ gens,
                                                                             const DevTile *__restrict__ tiles,
                                                                             const unsigned *__restrict__ runs,
                                                                             const unsigned *__restrict__ bounds,
                                                                             unsigned *counters, int ntiles)
{
    __shared__ WaveStage stage[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *mk = reinterpret_cast<uint32_t *>(&stage[wave]);
    QueueCursor cursor;
    for (int pass = 0;; pass++) {
        int t = 0;
        if constexpr (DIRECT) {
            t = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WAVES + wave);
            if (pass > 0 || t >= ntiles)
                break;
        } else {
            if (lane == 0)
                t = queue_next_tile(counters, runs, bounds, cursor);
            t = __builtin_amdgcn_readlane(t, 0);
            if (t < 0)
                break;
        }
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
    if (!DIRECT && lane == 0)
        queue_retire(counters, gridDim.x * WAVES);
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
// A: the caller's LDS matrix, MAXN rows of inv_pitch<MAXN, DW>() dwords; row(r) gives the
// address of the matrix's row r (N bytes, device memory written before this kernel or
// read-only input).  DW: dwords of a row that one thread updates per pivot step, 1 (a
// 4-byte LDS access per row) or 4 (one 16-byte access, and one table lookup for the four).
template <int MAXN, int DW = 1>
constexpr int inv_pitch()
{
    // DW 1: odd, so a column's bytes spread over the banks; DW 4: 16-byte rows, 4 dwords apart
    return DW == 4 ? MAXN / 4 + 4 : MAXN / 4 + 1;
}

template <int MAXN, int NT = 256, int DW = 1, class RowOf>
__device__ void invert_rows(uint32_t *A, RowOf row, int N, uint8_t *__restrict__ Cinv, int *rank_out,
                            const uint4 *__restrict__ ptab4, const uint8_t *__restrict__ invg)
{
    static_assert(DW == 1 || DW == 4, "rows are updated a dword or 16 bytes at a time");
    constexpr int RW = MAXN / 4;   // dwords of a row
    constexpr int PRW = inv_pitch<MAXN, DW>();   // row stride in LDS, dwords
    __shared__ uint4 T[256][2];
    __shared__ uint8_t IV[256];
    __shared__ uint8_t fcol[MAXN];
    __shared__ int cand[4];
    __shared__ int piv[MAXN];
    __shared__ int src[MAXN];
    uint8_t *Ab = reinterpret_cast<uint8_t *>(A);
    // NT threads take part: the whole workgroup (256 or 1024, barriers between
    // the phases) or its first wave alone (64, which needs no workgroup barrier:
    // a wave's LDS accesses complete in order).
    static_assert(NT == 256 || NT == 512 || NT == 1024 || (NT == 64 && MAXN <= 64),
                  "invert_rows runs on 256, 512 or 1024 threads, or on 64 for N <= 64");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto sync = [&]() {
        if constexpr (NT >= 256)
            __syncthreads();
        else
            wave_sync();
    };
    const int NW = (N + 3) >> 2;
    // row updates: thread tid owns column dword cl of rows r0, r0 + RS, ... (DW = 4: the
    // column dwords 4 cl .. 4 cl + 3)
    constexpr int RS = NT / (RW / DW);
    const int cl = tid % (RW / DW), r0 = tid / (RW / DW);

    // all loads of a phase are issued before the first is used (one memory wait)
#pragma unroll
    for (int i = tid; i < 512; i += NT)
        T[i >> 1][i & 1] = ptab4[i];
#pragma unroll
    for (int i = tid; i < 256; i += NT)
        IV[i] = invg[i];

    auto load_matrix = [&]() {
#pragma unroll 4
        for (int i = tid; i < N * RW; i += NT) {
            const int r = i / RW, w = i - r * RW;
            const uint8_t *src = row(r);
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; b++) {   // clamped, masked: no branch between the loads
                const int c = 4 * w + b;
                const uint32_t x = src[min(c, N - 1)];
                v |= (c < N ? x : 0u) << (8 * b);
            }
            A[r * PRW + w] = v;
        }
    };
    // lowest row index >= from with a nonzero entry in column j (>= N if none)
    auto find_pivot = [&](int j, int from) -> int {
        const bool ok = tid < N && tid >= from && Ab[tid * (4 * PRW) + j] != 0;
        const uint64_t m = __ballot(ok);
        if constexpr (NT == 64)
            return m ? (int)__builtin_ctzll(m) : (1 << 30);
        if (lane == 0 && wave < 4)   // rows < 256 sit in the first four waves
            cand[wave] = m ? wave * 64 + __builtin_ctzll(m) : (1 << 30);
        sync();
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
    sync();

    // Two barriers per pivot in the usual case: (1) the pivot row is scaled
    // while every thread reads the factors of its rows from column j into
    // registers; (2) the rows are updated, their table lookups independent of
    // one another.  The pivot is row j itself when its entry in column j is
    // nonzero (a random matrix almost always has one); only otherwise is the
    // column searched and a lower row swapped in.
    constexpr int RPT = (MAXN + RS - 1) / RS;   // rows per thread
    bool singular = false;
    for (int j = 0; j < N; j++) {
        int pr = j;
        if (__builtin_amdgcn_readfirstlane((uint32_t)Ab[j * (4 * PRW) + j]) == 0) {
            pr = find_pivot(j, j + 1);
            if (pr >= N) {
                singular = true;
                break;
            }
            swap_rows(pr, j);
            sync();
        }
        if (tid == 0)
            piv[j] = pr;
        uint32_t f[RPT];
#pragma unroll
        for (int m = 0; m < RPT; m++) {
            const int i = r0 + m * RS;
            f[m] = (i < N && i != j) ? (uint32_t)Ab[i * (4 * PRW) + j] : 0u;
        }
        if (tid < NW) {   // wave 0 only: reads below happen before the write
            uint32_t a = A[j * PRW + tid];
            const uint32_t pinv = IV[Ab[j * (4 * PRW) + j]];
            if (tid == (j >> 2))
                a = (a & ~(0xFFu << (8 * (j & 3)))) | (1u << (8 * (j & 3)));
            A[j * PRW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        sync();
        if constexpr (DW == 1) {
            if (cl < NW) {   // thread: column dword cl of rows r0, r0 + RS, ...
                // branch-free: where f is 0 the row's byte j is 0 already and the
                // product is 0 (row j itself, whose f is 0, keeps its leading 1)
                const uint32_t pj = A[j * PRW + cl];
                const uint32_t keep = cl == (j >> 2) ? ~(0xFFu << (8 * (j & 3))) : 0xFFFFFFFFu;
#pragma unroll
                for (int m = 0; m < RPT; m++) {
                    const int i = r0 + m * RS;
                    if (i < N) {
                        const uint32_t k = i == j ? 0xFFFFFFFFu : keep;
                        A[i * PRW + cl] = (A[i * PRW + cl] & k) ^ prod4(T[f[m]][0], T[f[m]][1].x, pj);
                    }
                }
            }
        } else {
            if (4 * cl < NW) {   // thread: column dwords 4 cl .. 4 cl + 3 of rows r0, r0 + RS, ...
                uint4 *A4 = reinterpret_cast<uint4 *>(A);
                constexpr int P4 = PRW / 4;
                const uint4 pj = A4[j * P4 + cl];
                // the dword of column j, if it is one of this thread's, loses byte j
                const uint32_t kj = ~(0xFFu << (8 * (j & 3)));
                const int dj = (j >> 2) - 4 * cl;   // 0..3 when this thread holds it
                const uint4 keep = {dj == 0 ? kj : ~0u, dj == 1 ? kj : ~0u, dj == 2 ? kj : ~0u, dj == 3 ? kj : ~0u};
#pragma unroll
                for (int m = 0; m < RPT; m++) {
                    const int i = r0 + m * RS;
                    if (i < N) {
                        const uint4 t0 = T[f[m]][0];
                        const uint32_t t1 = T[f[m]][1].x;
                        uint4 a = A4[i * P4 + cl];
                        const bool own = i == j;
                        a.x = (a.x & (own ? ~0u : keep.x)) ^ prod4(t0, t1, pj.x);
                        a.y = (a.y & (own ? ~0u : keep.y)) ^ prod4(t0, t1, pj.y);
                        a.z = (a.z & (own ? ~0u : keep.z)) ^ prod4(t0, t1, pj.z);
                        a.w = (a.w & (own ? ~0u : keep.w)) ^ prod4(t0, t1, pj.w);
                        A4[i * P4 + cl] = a;
                    }
                }
            }
        }
        sync();
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
        sync();
        for (int it = tid; it < N * N; it += NT) {
            const int i = it / N, c = it - i * N;
            Cinv[it] = Ab[i * (4 * PRW) + src[c]];
        }
        if (tid == 0 && rank_out)
            *rank_out = N;
        return;
    }

    // Singular: recompute the exact rank by forward elimination of a fresh copy.
    sync();
    load_matrix();
    sync();
    int prow = 0;
    for (int j = 0; j < N && prow < N; j++) {
        const int pr = find_pivot(j, prow);
        if (pr >= N) {
            sync();
            continue;
        }
        swap_rows(pr, prow);
        sync();
        if (tid < NW) {
            const uint32_t pinv = IV[Ab[prow * (4 * PRW) + j]];
            const uint32_t a = A[prow * PRW + tid];
            A[prow * PRW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        sync();
        if (tid < N)
            fcol[tid] = tid > prow ? Ab[tid * (4 * PRW) + j] : 0;
        sync();
        // a dword per thread here whatever DW is
        const int cw = tid % RW, rw0 = tid / RW;
        if (cw < NW) {
            const uint32_t pj = A[prow * PRW + cw];
#pragma unroll 4
            for (int i = rw0; i < N; i += NT / RW) {
                const uint32_t f = fcol[i];
                A[i * PRW + cw] ^= prod4(T[f][0], T[f][1].x, pj);
            }
        }
        sync();
        prow++;
    }
    if (tid == 0 && rank_out)
        *rank_out = prow;
}

// Gauss-Jordan inversion of the row-major N x N matrix at Cg.
template <int MAXN, int DW = 1>
__device__ void invert_body(const uint8_t *__restrict__ Cg, int N, uint8_t *__restrict__ Cinv, int *rank_out,
                            const uint4 *__restrict__ ptab4, const uint8_t *__restrict__ invg)
{
    __shared__ __align__(16) uint32_t A[MAXN * inv_pitch<MAXN, DW>()];
    invert_rows<MAXN, 256, DW>(A, [&](int r) { return Cg + (uint64_t)r * N; }, N, Cinv, rank_out, ptab4, invg);
}

// One matrix of more than 64 columns on 1024 threads: the pivot steps are
// latency-bound, and four times the waves hide more of it.
template <int MAXN, int DW = 1>
__global__ __launch_bounds__(1024) void k_invert_one_wide(const uint8_t *__restrict__ C, int N,
                                                          uint8_t *__restrict__ Cinv, int *rank,
                                                          const uint4 *__restrict__ ptab4,
                                                          const uint8_t *__restrict__ invg)
{
    __shared__ __align__(16) uint32_t A[MAXN * inv_pitch<MAXN, DW>()];
    invert_rows<MAXN, 1024, DW>(A, [&](int r) { return C + (uint64_t)r * N; }, N, Cinv, rank, ptab4, invg);
}

template <int MAXN, int DW = 1>
__global__ __launch_bounds__(256) void k_invert_one(const uint8_t *__restrict__ C, int N, uint8_t *__restrict__ Cinv,
                                                    int *rank, const uint4 *__restrict__ ptab4,
                                                    const uint8_t *__restrict__ invg)
{
    invert_body<MAXN, DW>(C, N, Cinv, rank, ptab4, invg);
}

// d_count (if not null): the number of systems in `sys`, known only on the
// device; workgroups past it have nothing to do.
template <int MAXN, int NT = 256, int DW = 1>
__global__ __launch_bounds__(NT) void k_invert_batched(const DevSys *__restrict__ sys,
                                                       const uint4 *__restrict__ ptab4,
                                                       const uint8_t *__restrict__ invg,
                                                       const unsigned *__restrict__ d_count)
{
    if (d_count && blockIdx.x >= *d_count)
        return;
    const DevSys s = sys[blockIdx.x];
    if ((int)s.N > MAXN || (MAXN > 32 && (int)s.N <= MAXN / 2))
        return;   // handled by the launch of another size class
    __shared__ __align__(16) uint32_t A[MAXN * inv_pitch<MAXN, DW>()];
    invert_rows<MAXN, NT, DW>(A, [&](int r) { return s.C + (uint64_t)r * s.N; }, (int)s.N, s.Cinv, s.rank, ptab4,
                              invg);
}

// ------------------------------------------------- one small generation
//
// A single small generation (N, K <= 32, short rows) is latency-bound: the
// general path streams the sources through a few waves one pair at a time
// and needs a second launch to clear the output of source slices.  Here one
// launch gives every (coded row, 4-byte column) its own thread, which issues
// all N source loads before anything else, so the kernel waits for memory
// about once; the K x N product tables are staged in LDS meanwhile.  For a
// decode the first wave of every workgroup also inverts C in its LDS (the
// Gauss-Jordan of k_invert_one, with wave barriers in place of workgroup
// ones) while the source loads are in flight, and all apply C^-1;
// workgroup 0 reports the rank, and a singular C writes no output.

constexpr int SMALL_MAX = 32;   // largest N and K of the small path
constexpr int REG_INV_MAX = 16;  // largest N inverted in one wave's registers

// Gauss-Jordan inversion of an N x N matrix, N <= 16, in one wave's registers:
// lane 4r + q holds bytes 4q .. 4q + 3 of row r.  At pivot step j a ballot
// over the lanes that hold column j finds the lowest usable row, a cross-lane
// permute swaps it up, the pivot row (its pivot replaced by 1) is multiplied
// by the pivot's inverse (TI: the field's product tables indexed by the
// element whose inverse they multiply by), and every other row takes its
// factor (its byte j) and the pivot row's dword from the lanes that hold them
// (cross-lane permutes) and clears column j.  (Taking them with a DPP quad
// broadcast and four scalar lane reads instead measured slower.)  The row
// swaps are undone as column swaps when the inverse is written to Ci (N x N,
// row-major, LDS).  W (64 dwords) and P (16 ints) are LDS scratch.  Returns N,
// or -1 when C is singular (Ci then unspecified).
__device__ int invert_wave_regs(const uint8_t *__restrict__ C, int N, uint8_t *Ci, const uint4 (*T)[2],
                                const uint4 (*TI)[2], uint32_t *W, int *P)
{
    const int lane = threadIdx.x & 63, r = lane >> 2, q = lane & 3;
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; b++) {   // clamped into the matrix, masked past it
        const int c = 4 * q + b;
        const uint32_t x = C[min(r, N - 1) * N + min(c, N - 1)];
        v |= (r < N && c < N ? x : 0u) << (8 * b);
    }
#pragma unroll
    for (int j = 0; j < REG_INV_MAX; j++) {
        if (j >= N)
            break;
        const int qj = j >> 2, sh = 8 * (j & 3);
        const uint64_t cand = __ballot(q == qj && r >= j && r < N && ((v >> sh) & 0xFFu) != 0);
        if (cand == 0)
            return -1;
        const int pr = __builtin_amdgcn_readfirstlane((int)(__builtin_ctzll(cand) >> 2));
        if (pr != j) {
            const int src = r == j ? pr * 4 + q : r == pr ? j * 4 + q : lane;
            v = (uint32_t)__shfl((int)v, src);
        }
        if (lane == 0)
            P[j] = pr;
        const uint32_t p = ((uint32_t)__builtin_amdgcn_readlane((int)v, j * 4 + qj) >> sh) & 0xFFu;
        const uint32_t f = ((uint32_t)__shfl((int)v, r * 4 + qj) >> sh) & 0xFFu;   // this row's factor
        uint32_t vj = q == qj ? ((v & ~(0xFFu << sh)) | (1u << sh)) : v;
        vj = prod4(TI[p][0], TI[p][1].x, vj);
        const uint32_t pj = (uint32_t)__shfl((int)vj, j * 4 + q);   // the scaled pivot row's dword q
        const uint32_t keep = q == qj ? ~(0xFFu << sh) : 0xFFFFFFFFu;
        v = r == j ? vj : ((v & keep) ^ prod4(T[f][0], T[f][1].x, pj));
    }
    W[lane] = v;
    wave_sync();
    for (int e = lane; e < N * N; e += 64) {
        const int i = e / N, c = e - i * N;
        int x = c;   // the column of the eliminated matrix that holds column c of the inverse
        for (int l = 0; l < N; l++) {
            const int pl = P[l];
            x = x == l ? pl : x == pl ? l : x;
        }
        Ci[e] = (uint8_t)(W[i * 4 + (x >> 2)] >> (8 * (x & 3)));
    }
    return N;
}

__global__ __launch_bounds__(256) void k_small(const uint8_t *__restrict__ C, int K, int N,
                                               const uint8_t *__restrict__ S, uint64_t ld_s, uint8_t *__restrict__ Y,
                                               uint64_t ld_y, uint64_t len, const uint4 *__restrict__ ptab4,
                                               const uint4 *__restrict__ ptabinv4, const uint8_t *__restrict__ invg,
                                               int *rank, int decode)
{
    __shared__ uint4 T[SMALL_MAX * SMALL_MAX][2];
    __shared__ uint8_t Ci[SMALL_MAX * SMALL_MAX];
    __shared__ int rk;
    const uint64_t ncols = (len + 3) / 4;
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t kq = t / ncols;
    const bool active = kq < (uint64_t)K;   // threads past the last row still join the barriers
    const int k = active ? (int)kq : 0;
    const uint64_t col = 4 * (t - kq * ncols);
    const uint64_t avail = active ? len - col : 0;
    // every source load is issued before the first is used: rows past N read
    // row N - 1 (in bounds) and are masked to zero, with no branch per row
    uint32_t x[SMALL_MAX];
    if (avail >= 4) {
#pragma unroll
        for (int i = 0; i < SMALL_MAX; i++) {
            const uint32_t v = gld<uint32_t>(S + (uint64_t)min(i, N - 1) * ld_s + col);
            x[i] = i < N ? v : 0u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < SMALL_MAX; i++) {
            x[i] = 0;
            if (i < N)
                for (uint64_t b = 0; b < avail; b++)
                    x[i] |= (uint32_t)gld<uint8_t>(S + (uint64_t)i * ld_s + col + b) << (8 * b);
        }
    }
    const uint8_t *coef = C;
    __shared__ uint4 FT[256][2], FTI[256][2];   // the field's product tables, and those of the inverses
    const bool regs = decode && N <= REG_INV_MAX;
    if (regs) {   // every thread fetches two of each
        for (int e = threadIdx.x; e < 512; e += 256) {
            FT[e >> 1][e & 1] = ptab4[e];
            FTI[e >> 1][e & 1] = ptabinv4[e];
        }
        __syncthreads();
    }
    if (decode) {
        __shared__ __align__(16) uint32_t A[SMALL_MAX * inv_pitch<SMALL_MAX, 4>()];
        __shared__ uint32_t W[64];
        __shared__ int P[REG_INV_MAX];
        if (threadIdx.x < 64) {   // one wave: no workgroup barrier per pivot
            int got = -1;
            if (regs)
                got = invert_wave_regs(C, N, Ci, FT, FTI, W, P);
            if (got < 0)   // larger, or singular: the LDS elimination, which also finds the rank
                invert_rows<SMALL_MAX, 64, 4>(A, [&](int r) { return C + (uint64_t)r * N; }, N, Ci, &rk, ptab4,
                                              invg);
            else if (threadIdx.x == 0)
                rk = got;
        }
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0 && rank)
            *rank = rk;
        if (rk < N)
            return;   // the same value in every thread of the workgroup
        coef = Ci;
    }
    for (int e = threadIdx.x; e < K * N; e += 256) {
        const uint32_t c = coef[e];
        T[e][0] = regs ? FT[c][0] : ptab4[c * 2];   // from the LDS copy when there is one
        T[e][1] = regs ? FT[c][1] : ptab4[c * 2 + 1];
    }
    __syncthreads();
    if (avail == 0)
        return;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < SMALL_MAX; i++)
        if (i < N)
            acc ^= prod4(T[k * N + i][0], T[k * N + i][1].x, x[i]);
    uint8_t *q = Y + (uint64_t)k * ld_y + col;
    if (avail >= 4)
        gst<uint32_t>(q, acc);
    else
        for (uint64_t b = 0; b < avail; b++)
            gst<uint8_t>(q + b, (uint8_t)(acc >> (8 * b)));
}

// ------------------------------------------------------------------ serving

// Progressive decoding of one generation (one workgroup per generation).
// The innovative coefficient vectors received so far are kept in reduced row
// echelon form R, together with the transform T that produced it from the
// accepted packets' raw vectors Csel (R = T Csel; row j of T has weights on the
// packets accepted so far).  An arriving vector c is reduced against R in one
// pass: since every row of R is zero in the other rows' pivot columns,
// subtracting c[pivot(r)] * R[r] for all r at once clears every pivot column,
// and the same multiples of T's rows (plus the unit weight of the new packet)
// give its transform row t.  If nothing is left of c the packet carried no new
// information.  Otherwise c and t are scaled to a leading 1, c's pivot column
// is cleared from R (T's rows take the same updates), and the payload is
// stored.  At rank N, R is the identity with its rows in pivot order, so
// row pivot(j) of Csel^-1 is row j of T: the kernel writes Csel^-1 directly and
// the step's payload product S = Csel^-1 * Bsel needs no separate inversion.
//
// During a step R and T live in LDS; the packets are taken ABSORB_PKC at a
// time, their descriptors and coefficient vectors loaded into LDS together, so
// the loop over packets touches device memory only at those refills.  A
// packet costs three workgroup barriers (two when it is dropped): every wave
// reduces the vector against its share of R's rows and XORs its partial sums
// into one LDS accumulator with atomics; wave 0 alone finds the leading entry
// and scales the row, and after its share of clearing the new pivot column
// from R sets up the next packet's accumulator.  The innovative packets'
// payloads are copied out after the loop.
constexpr int ABSORB_PKC = 32;

// One workgroup per generation of 16 waves: the passes over R of each packet
// split its rows 16 ways (a step has at most a few dozen such workgroups, so
// each has a CU to itself).
constexpr int ABSORB_THREADS = 1024, ABSORB_WAVES = ABSORB_THREADS / 64;

__global__ __launch_bounds__(ABSORB_THREADS) void k_absorb(const DevAbsorb *__restrict__ items,
                                                const DevPacket *__restrict__ pkts, const uint4 *__restrict__ ptab4,
                                                const uint8_t *__restrict__ invg)
{
    __shared__ uint32_t Rl[256 * 65];   // row r at Rl + 65 r (odd stride)
    __shared__ uint32_t Tl[256 * 65];   // transform rows, the same layout
    __shared__ uint32_t cw[64], tw[64];   // the accepted packet's scaled vector and transform row
    __shared__ uint32_t xacc[64], tacc[64];   // the current packet's reduction, summed by atomics
    __shared__ uint32_t coefs[ABSORB_PKC][64];   // coefficient dwords of the cached packets
    __shared__ uint4 TB[256][2];
    __shared__ uint8_t IV[256];
    __shared__ int pivc[256];
    __shared__ const uint8_t *row_pay[256];   // payloads of the rows added in this step
    __shared__ const uint8_t *pay_c[ABSORB_PKC];
    __shared__ int s_lead;
    const DevAbsorb it = items[blockIdx.x];
    const DevDecSlot &s = it.s;
    const int N = (int)s.N, NW = (N + 3) >> 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint8_t *Rb = reinterpret_cast<const uint8_t *>(Rl);   // row r at byte 260 r
    const uint8_t *Tb = reinterpret_cast<const uint8_t *>(Tl);

    int rank = s.meta[0];
    if (rank >= N || N > 256)
        return;
    const int rank0 = rank;
    for (int i = tid; i < 512; i += ABSORB_THREADS)
        TB[i >> 1][i & 1] = ptab4[i];
    if (tid < 256)
        IV[tid] = invg[tid];
    for (int i = tid; i < rank; i += ABSORB_THREADS)
        pivc[i] = s.meta[4 + i];
    for (int i = tid; i < rank * NW; i += ABSORB_THREADS) {
        const int r = i / NW, w = i - r * NW;
        Rl[r * 65 + w] = reinterpret_cast<const uint32_t *>(s.R + (uint64_t)r * s.rs)[w];
        Tl[r * 65 + w] = reinterpret_cast<const uint32_t *>(s.T + (uint64_t)r * s.rs)[w];
    }
    // descriptors and coefficient vectors of packets q0 .. q0 + ABSORB_PKC - 1 (dword w of
    // packet p at coefs[p][w], bytes past N zero); ends with a barrier
    auto refill = [&](uint32_t q0) {
        for (int e = tid; e < ABSORB_PKC * 64; e += ABSORB_THREADS) {
            const int p = e >> 6, w = e & 63;
            uint32_t v = 0;
            if (q0 + p < it.npk && w < NW) {
                const uint8_t *c = pkts[it.pk0 + q0 + p].coef;
#pragma unroll
                for (int b = 0; b < 4; b++)
                    if (4 * w + b < N)
                        v |= (uint32_t)c[4 * w + b] << (8 * b);
            }
            coefs[p][w] = v;
        }
        if (tid < ABSORB_PKC && q0 + tid < it.npk)
            pay_c[tid] = pkts[it.pk0 + q0 + tid].payload;
        __syncthreads();
    };
    // wave 0: the reduction of packet slot p starts from its own vector and,
    // in the transform, its unit weight at the next row's index
    auto start_packet = [&](int p) {
        if (wave == 0) {
            xacc[lane] = coefs[p][lane];
            tacc[lane] = lane == (rank >> 2) ? 1u << (8 * (rank & 3)) : 0u;
        }
    };
    int seen = 0, dropped = 0;
    if (it.npk > 0) {
        refill(0);
        start_packet(0);
        __syncthreads();
    }

    for (uint32_t q = 0; q < it.npk && rank < N; q++) {
        const int slot = (int)(q % ABSORB_PKC);
        // wave w sums rows w, w + W, ... of column dword `lane`, in R and in T; the
        // factor of a row is the vector's entry in the row's pivot column (zero
        // factors add zero products)
        if (lane < NW) {
            uint32_t acc = 0, tac = 0;
#pragma unroll 4
            for (int r = wave; r < rank; r += ABSORB_WAVES) {
                const int pc = pivc[r];
                const uint32_t f = (coefs[slot][pc >> 2] >> (8 * (pc & 3))) & 0xFFu;
                acc ^= prod4(TB[f][0], TB[f][1].x, Rl[r * 65 + lane]);
                tac ^= prod4(TB[f][0], TB[f][1].x, Tl[r * 65 + lane]);
            }
            if (acc)
                atomicXor(&xacc[lane], acc);
            if (tac)
                atomicXor(&tacc[lane], tac);
        }
        __syncthreads();
        if (wave == 0) {   // leading entry, then the row scaled to a leading 1
            uint32_t x = lane < NW ? xacc[lane] : 0u, t = lane < NW ? tacc[lane] : 0u;
            const uint64_t m = __ballot(x != 0);
            int lead = N;
            if (m) {
                const int l0 = (int)__builtin_ctzll(m);
                const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)x, l0);
                lead = 4 * l0 + (int)(__builtin_ctz(x0) >> 3);
                const uint32_t iv = IV[(x0 >> (8 * (lead & 3))) & 0xFFu];
                x = prod4(TB[iv][0], TB[iv][1].x, x);
                t = prod4(TB[iv][0], TB[iv][1].x, t);
                if (lane < NW) {
                    cw[lane] = x;
                    tw[lane] = t;
                }
            }
            if (lane == 0)
                s_lead = lead;
        }
        __syncthreads();
        const int lead = s_lead;
        seen++;
        const bool next_cached = slot + 1 < ABSORB_PKC && q + 1 < it.npk;
        if (lead >= N) {   // nothing new in this packet
            dropped++;
            if (next_cached) {
                start_packet(slot + 1);
                __syncthreads();
            } else if (q + 1 < it.npk) {
                refill(q + 1);
                start_packet(0);
                __syncthreads();
            }
            continue;
        }
        if (lane < NW) {   // wave w clears the new pivot column from rows w, w + W, ... (T alike)
            const uint32_t c = cw[lane], t = tw[lane];
#pragma unroll 4
            for (int r = wave; r < rank; r += ABSORB_WAVES) {
                const uint32_t f = Rb[r * 260 + lead];   // read by the whole wave before its row changes
                Rl[r * 65 + lane] ^= prod4(TB[f][0], TB[f][1].x, c);
                Tl[r * 65 + lane] ^= prod4(TB[f][0], TB[f][1].x, t);
            }
        }
        if (tid < NW) {
            Rl[rank * 65 + tid] = cw[tid];
            Tl[rank * 65 + tid] = tw[tid];
        }
        if (tid == 0) {
            pivc[rank] = lead;
            row_pay[rank] = pay_c[slot];
        }
        rank++;
        if (next_cached)
            start_packet(slot + 1);
        __syncthreads();
        if (!next_cached && q + 1 < it.npk && rank < N) {
            refill(q + 1);
            start_packet(0);
            __syncthreads();
        }
    }
    // R and T back to device memory; the new rows' payloads
    for (int i = tid; i < rank * NW; i += ABSORB_THREADS) {
        const int r = i / NW, w = i - r * NW;
        reinterpret_cast<uint32_t *>(s.R + (uint64_t)r * s.rs)[w] = Rl[r * 65 + w];
        reinterpret_cast<uint32_t *>(s.T + (uint64_t)r * s.rs)[w] = Tl[r * 65 + w];
    }
    for (int rr = rank0; rr < rank; rr++) {
        const uint8_t *src = row_pay[rr];
        uint8_t *dst = s.Bsel + (uint64_t)rr * s.ld;
        if (((((uintptr_t)dst) | ((uintptr_t)src)) & 3u) == 0) {
            const uint64_t words = s.len >> 2;
            for (uint64_t w = tid; w < words; w += ABSORB_THREADS)
                reinterpret_cast<uint32_t *>(dst)[w] = reinterpret_cast<const uint32_t *>(src)[w];
            for (uint64_t b = (words << 2) + tid; b < s.len; b += ABSORB_THREADS)
                dst[b] = src[b];
        } else {
            for (uint64_t b = tid; b < s.len; b += ABSORB_THREADS)
                dst[b] = src[b];
        }
    }
    for (int i = tid; i < rank; i += ABSORB_THREADS)
        s.meta[4 + i] = pivc[i];
    if (rank == N) {   // complete: row pivot(j) of Csel^-1 is row j of T
        for (int i = tid; i < N * N; i += ABSORB_THREADS) {
            const int j = i / N, b = i - j * N;
            s.Cinv[(uint64_t)pivc[j] * N + b] = Tb[j * 260 + b];
        }
    }
    if (tid == 0) {
        s.meta[0] = rank;
        s.meta[2] += seen;
        s.meta[3] += dropped;
        if (rank == N)
            s.meta[1] = it.step;   // releases the step's payload product for this generation
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
    // a block per 8 KiB, all at once (two 16-byte pieces per thread): on a
    // 1 GiB region 1.79 TB/s of x against 1.51 for a grid capped at 4096
    // blocks that loops over the region
    uint64_t blocks = (len / 16 + 511) / 512;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
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
    if (max_len >= REGION_CHUNK) {
        // long regions: a block per 4 KiB chunk keeps the descriptor and tables uniform
        const uint64_t gx = (max_len + REGION_CHUNK - 1) / REGION_CHUNK;
        if (gx > 0x7FFFFFFFull)
            return hipErrorInvalidValue;
        for (int base = 0; base < count; base += 65535) {   // grid.y is limited to 65535
            const int n = min(65535, count - base);
            hipLaunchKernelGGL(k_region_chunks, dim3((unsigned)gx, (unsigned)n), dim3(256), 0, s,
                               reinterpret_cast<const RegionDesc *>(d_regions) + base,
                               reinterpret_cast<const uint4 *>(ptab_field), q);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    // shorter regions: a wave each, M 1024-byte rounds per lane
    const int M = (int)((max_len + 1023) / 1024);
    // a wave per region, all at once: measured faster than a persistent
    // grid of two, four or eight workgroups per CU (the dispatcher keeps the
    // CUs fed, and no wave's loads queue behind its previous region's stores)
    const unsigned blocks = (unsigned)(((uint64_t)count + REGION_WAVES - 1) / REGION_WAVES);
    const RegionDesc *r = reinterpret_cast<const RegionDesc *>(d_regions);
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    if (M <= 1)
        hipLaunchKernelGGL(k_region_waves<1>, dim3(blocks), dim3(256), 0, s, r, pt, q, count);
    else if (M == 2)
        hipLaunchKernelGGL(k_region_waves<2>, dim3(blocks), dim3(256), 0, s, r, pt, q, count);
    else if (M == 3)
        hipLaunchKernelGGL(k_region_waves<3>, dim3(blocks), dim3(256), 0, s, r, pt, q, count);
    else
        hipLaunchKernelGGL(k_region_waves<4>, dim3(blocks), dim3(256), 0, s, r, pt, q, count);
    return hipGetLastError();
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

bool small_ok(int K, int N, uint64_t len, uint32_t align)
{
    return K >= 1 && K <= SMALL_MAX && N >= 1 && N <= SMALL_MAX && len >= 1 && len <= 8192 && align >= 4;
}

hipError_t launch_small(const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s, uint8_t *Y, uint64_t ld_y,
                        uint64_t len, const uint32_t *ptab_field, const uint32_t *ptab_inv_field,
                        const uint8_t *inv_field, int *rank, bool decode, hipStream_t s)
{
    if (!small_ok(K, N, len, 4))
        return hipErrorInvalidValue;
    const uint64_t threads = (len + 3) / 4 * (uint64_t)K;
    hipLaunchKernelGGL(k_small, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, C, K, N, S, ld_s, Y, ld_y,
                       len, reinterpret_cast<const uint4 *>(ptab_field), reinterpret_cast<const uint4 *>(ptab_inv_field),
                       inv_field, rank, decode ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_encode_persistent(const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                    const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                    const uint32_t *ptab_field, hipStream_t s, bool direct)
{
    if (ntiles <= 0)
        return hipSuccess;
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    if (direct)
        hipLaunchKernelGGL(k_encode_waves<true>, dim3((unsigned)((ntiles + WAVES - 1) / WAVES)), dim3(256), 0, s,
                           gens, tiles, runs, bounds, counters, pt, ntiles);
    else
        hipLaunchKernelGGL(k_encode_waves<false>, dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters,
                           pt, ntiles);
    return hipGetLastError();
}

template <int NB>
static void launch_planes_nb(const DevGen *gens, const DevTile *tiles, const unsigned *runs, const unsigned *bounds,
                             int ntiles, unsigned *counters, int grid, hipStream_t s, bool direct)
{
    if (direct)
        hipLaunchKernelGGL((k_encode_planes<NB, true>), dim3((unsigned)((ntiles + WAVES - 1) / WAVES)), dim3(256), 0,
                           s, gens, tiles, runs, bounds, counters, ntiles);
    else
        hipLaunchKernelGGL((k_encode_planes<NB, false>), dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds,
                           counters, ntiles);
}

hipError_t launch_encode_planes(int field, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid, hipStream_t s,
                                bool direct)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (field == 1)
        launch_planes_nb<1>(gens, tiles, runs, bounds, ntiles, counters, grid, s, direct);
    else if (field == 2)
        launch_planes_nb<2>(gens, tiles, runs, bounds, ntiles, counters, grid, s, direct);
    else if (field == 4)
        launch_planes_nb<4>(gens, tiles, runs, bounds, ntiles, counters, grid, s, direct);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// The streaming kernel for the batch's largest K or N (sk = 1, 2, 4 or 8).
static const void *stream_kernel(int sk)
{
    return sk <= 1   ? reinterpret_cast<const void *>(&k_encode_stream<1, 8>)
           : sk <= 2 ? reinterpret_cast<const void *>(&k_encode_stream<2, 4>)
           : sk <= 4 ? reinterpret_cast<const void *>(&k_encode_stream<4, 2>)
                     : reinterpret_cast<const void *>(&k_encode_stream<8, 1>);
}

hipError_t launch_encode_stream(int sk, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                const uint32_t *ptab_field, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    if (sk <= 1)
        hipLaunchKernelGGL((k_encode_stream<1, 8>), dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters, pt);
    else if (sk <= 2)
        hipLaunchKernelGGL((k_encode_stream<2, 4>), dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters, pt);
    else if (sk <= 4)
        hipLaunchKernelGGL((k_encode_stream<4, 2>), dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters, pt);
    else
        hipLaunchKernelGGL((k_encode_stream<8, 1>), dim3(grid), dim3(256), 0, s, gens, tiles, runs, bounds, counters, pt);
    return hipGetLastError();
}

int encode_chunks_strips(int sk)
{
    return sk <= 1 ? 8 : sk <= 2 ? 4 : sk <= 4 ? 2 : 1;
}

hipError_t launch_encode_chunks(int sk, const DevGen *gens, const DevTile *tiles, int ntiles,
                                const uint32_t *ptab_field, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    const dim3 grid((unsigned)((ntiles + WAVES - 1) / WAVES));
    if (sk <= 1)
        hipLaunchKernelGGL((k_encode_chunks<1, 8>), grid, dim3(256), 0, s, gens, tiles, ntiles, pt);
    else if (sk <= 2)
        hipLaunchKernelGGL((k_encode_chunks<2, 4>), grid, dim3(256), 0, s, gens, tiles, ntiles, pt);
    else if (sk <= 4)
        hipLaunchKernelGGL((k_encode_chunks<4, 2>), grid, dim3(256), 0, s, gens, tiles, ntiles, pt);
    else
        hipLaunchKernelGGL((k_encode_chunks<8, 1>), grid, dim3(256), 0, s, gens, tiles, ntiles, pt);
    return hipGetLastError();
}

int encode_stream_blocks_per_cu(int sk)
{
    static int cached[4] = {0, 0, 0, 0};
    const int ix = sk <= 1 ? 0 : sk <= 2 ? 1 : sk <= 4 ? 2 : 3;
    if (cached[ix] > 0)
        return cached[ix];
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream_kernel(sk), 256, 0) != hipSuccess || nb < 1)
        return 1;
    cached[ix] = nb;
    return nb;
}

int encode_planes_blocks_per_cu(int field)
{
    const void *k = field == 1   ? reinterpret_cast<const void *>(&k_encode_planes<1, false>)
                    : field == 2 ? reinterpret_cast<const void *>(&k_encode_planes<2, false>)
                                 : reinterpret_cast<const void *>(&k_encode_planes<4, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess || nb < 1)
        return 1;
    return nb;
}

int encode_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_encode_waves<false>), 256, 0) !=
            hipSuccess ||
        nb < 1)
        return 1;
    return nb;
}

hipError_t launch_invert(const DevSys *sys, int count, const uint8_t *C, int N, uint8_t *Cinv, int *rank,
                         const uint32_t *ptab_field, const uint8_t *inv_field, hipStream_t s,
                         const unsigned *d_count)
{
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
    if (sys == nullptr) {   // 16 bytes per thread per row update: 256 x 256 in 0.44 ms instead of 0.65
        if (N <= 32)
            hipLaunchKernelGGL((k_invert_one<32, 4>), dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        else if (N <= 64)
            hipLaunchKernelGGL((k_invert_one<64, 4>), dim3(1), dim3(256), 0, s, C, N, Cinv, rank, pt, inv_field);
        else if (N <= 128)
            hipLaunchKernelGGL((k_invert_one_wide<128, 4>), dim3(1), dim3(1024), 0, s, C, N, Cinv, rank, pt, inv_field);
        else
            hipLaunchKernelGGL((k_invert_one_wide<256, 4>), dim3(1), dim3(1024), 0, s, C, N, Cinv, rank, pt, inv_field);
        return hipGetLastError();
    }
    if (count <= 0)
        return hipSuccess;
    // `sys` holds systems of one size class (the class of N); a block skips any other.  Rows
    // are updated 16 bytes per thread (measured 4% faster on a 2,048-system decode than 4).
    if (N <= 32)
        hipLaunchKernelGGL((k_invert_batched<32, 256, 4>), dim3(count), dim3(256), 0, s, sys, pt, inv_field, d_count);
    else if (N <= 64)
        hipLaunchKernelGGL((k_invert_batched<64, 256, 4>), dim3(count), dim3(256), 0, s, sys, pt, inv_field, d_count);
    else if (N <= 128)
        hipLaunchKernelGGL((k_invert_batched<128, 256, 4>), dim3(count), dim3(256), 0, s, sys, pt, inv_field, d_count);
    else
        hipLaunchKernelGGL((k_invert_batched<256, 256, 4>), dim3(count), dim3(256), 0, s, sys, pt, inv_field, d_count);
    return hipGetLastError();
}

hipError_t launch_absorb(const DevAbsorb *items, int n, const DevPacket *pkts, const uint32_t *ptab_field,
                         const uint8_t *inv_field, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_absorb, dim3(n), dim3(ABSORB_THREADS), 0, s, items, pkts,
                       reinterpret_cast<const uint4 *>(ptab_field), inv_field);
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

}  // namespace gfnc
