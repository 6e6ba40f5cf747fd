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

template <int D>
__device__ __forceinline__ void load_row(const uint8_t *p, uint64_t avail, bool vec, uint32_t (&x)[D])
{
    if (vec && avail >= 4u * D) {
        if constexpr (D == 4) {
            const uint4 t = *reinterpret_cast<const uint4 *>(p);
            x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
        } else if constexpr (D == 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            x[0] = t.x; x[1] = t.y;
        } else {
            x[0] = *reinterpret_cast<const uint32_t *>(p);
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; d++)
            x[d] = 0;
#pragma unroll
        for (int b = 0; b < 4 * D; b++)
            if ((uint64_t)b < avail)
                x[b >> 2] |= (uint32_t)p[b] << (8 * (b & 3));
    }
}

template <int D>
__device__ __forceinline__ void store_row(uint8_t *p, uint64_t avail, bool vec, const uint32_t (&x)[D])
{
    if (vec && avail >= 4u * D) {
        if constexpr (D == 4) {
            *reinterpret_cast<uint4 *>(p) = make_uint4(x[0], x[1], x[2], x[3]);
        } else if constexpr (D == 2) {
            *reinterpret_cast<uint2 *>(p) = make_uint2(x[0], x[1]);
        } else {
            *reinterpret_cast<uint32_t *>(p) = x[0];
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4 * D; b++)
            if ((uint64_t)b < avail)
                p[b] = (uint8_t)(x[b >> 2] >> (8 * (b & 3)));
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

// One tile: KW coded rows (k0 ...) x one block strip of 4 waves * 64 lanes *
// 4D bytes starting at p0.  Every thread of the block must call this.
template <int D, int KW>
__device__ __forceinline__ void enc_tile(const uint8_t *__restrict__ C, int K, int N,
                                         const uint8_t *__restrict__ S, uint64_t ld_s, uint8_t *__restrict__ Y,
                                         uint64_t ld_y, uint64_t len, int k0, uint64_t p0, bool vec,
                                         const uint4 *__restrict__ ptab4, uint4 (*tabs)[NC][2])
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint64_t p = p0 + (uint64_t)wave * (256u * D) + (uint64_t)lane * (4u * D);
    const bool active = p < len;
    const uint64_t avail = active ? len - p : 0;

    uint32_t acc[KW][D];
#pragma unroll
    for (int kk = 0; kk < KW; kk++)
#pragma unroll
        for (int d = 0; d < D; d++)
            acc[kk][d] = 0;

    for (int n0 = 0; n0 < N; n0 += NC) {
        const int nc = min(NC, N - n0);
        __syncthreads();
        for (int idx = tid; idx < KW * NC; idx += 256) {
            const int kk = idx / NC, nn = idx % NC;
            const int k = k0 + kk;
            const uint32_t c = (k < K && nn < nc) ? (uint32_t)C[(uint64_t)k * N + n0 + nn] : 0u;
            tabs[kk][nn][0] = ptab4[c * 2];
            tabs[kk][nn][1] = ptab4[c * 2 + 1];
        }
        __syncthreads();
        if (active) {
            const uint8_t *src = S + (uint64_t)n0 * ld_s + p;
            uint32_t xn[D];
            load_row<D>(src, avail, vec, xn);
            for (int nn = 0; nn < nc; nn++) {
                uint32_t x[D];
#pragma unroll
                for (int d = 0; d < D; d++)
                    x[d] = xn[d];
                if (nn + 1 < nc)
                    load_row<D>(src + (uint64_t)(nn + 1) * ld_s, avail, vec, xn);
                Sel s[D];
#pragma unroll
                for (int d = 0; d < D; d++)
                    s[d] = split(x[d]);
#pragma unroll
                for (int kk = 0; kk < KW; kk++) {
                    const uint4 ta = tabs[kk][nn][0];
                    const uint32_t tb = tabs[kk][nn][1].x;
#pragma unroll
                    for (int d = 0; d < D; d++)
                        acc[kk][d] ^= prod(ta.x, ta.y, ta.z, ta.w, tb, s[d]);
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int kk = 0; kk < KW; kk++)
            if (k0 + kk < K)
                store_row<D>(Y + (uint64_t)(k0 + kk) * ld_y + p, avail, vec, acc[kk]);
    }
}

template <int D, int KW>
__global__ __launch_bounds__(256) void k_encode(const uint8_t *__restrict__ C, int K, int N,
                                                const uint8_t *__restrict__ S, uint64_t ld_s,
                                                uint8_t *__restrict__ Y, uint64_t ld_y, uint64_t len,
                                                const uint4 *__restrict__ ptab4, const int *__restrict__ status,
                                                int need, int vec)
{
    __shared__ uint4 tabs[KW][NC][2];
    if (status && *status != need)
        return;
    enc_tile<D, KW>(C, K, N, S, ld_s, Y, ld_y, len, (int)blockIdx.y * KW,
                    (uint64_t)blockIdx.x * (1024u * D), vec != 0, ptab4, tabs);
}

// Persistent encode over a tile list.  counters[0] hands out tiles,
// counters[1] counts retired blocks; the last block to retire resets both so
// the next launch (or graph replay) starts from zero without a memset.
template <int D, int KW>
__global__ __launch_bounds__(256) void k_encode_persistent(const DevGen *__restrict__ gens,
                                                           const DevTile *__restrict__ tiles, int ntiles,
                                                           unsigned *counters, const uint4 *__restrict__ ptab4)
{
    __shared__ uint4 tabs[KW][NC][2];
    __shared__ int s_tile;
    for (;;) {
        if (threadIdx.x == 0)
            s_tile = (int)atomicAdd(&counters[0], 1u);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= ntiles)
            break;
        const DevTile tl = tiles[t];
        const DevGen g = gens[tl.gen];
        if (g.status && *g.status != g.need)
            continue;
        enc_tile<D, KW>(g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, (int)tl.k0, tl.p0,
                        g.aligned != 0, ptab4, tabs);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
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
template <int MAXN>
__device__ void invert_body(const uint8_t *__restrict__ Cg, int N, uint8_t *__restrict__ Cinv, int *rank_out,
                            const uint4 *__restrict__ ptab4, const uint8_t *__restrict__ invg)
{
    constexpr int RW = MAXN / 4;   // dwords per row
    __shared__ uint32_t A[MAXN * RW];
    __shared__ uint4 T[256][2];
    __shared__ uint8_t IV[256];
    __shared__ uint8_t fcol[MAXN];
    __shared__ int cand[4];
    __shared__ int piv[MAXN];
    __shared__ int src[MAXN];
    uint8_t *Ab = reinterpret_cast<uint8_t *>(A);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NW = (N + 3) >> 2;

    for (int i = tid; i < 512; i += 256)
        T[i >> 1][i & 1] = ptab4[i];
    IV[tid] = invg[tid];

    auto load_matrix = [&]() {
        for (int i = tid; i < N * RW; i += 256) {
            const int r = i / RW, w = i - r * RW;
            uint32_t v = 0;
            for (int b = 0; b < 4; b++) {
                const int c = 4 * w + b;
                if (c < N)
                    v |= (uint32_t)Cg[(uint64_t)r * N + c] << (8 * b);
            }
            A[r * RW + w] = v;
        }
    };
    // lowest row index >= from with a nonzero entry in column j (>= N if none)
    auto find_pivot = [&](int j, int from) -> int {
        const bool ok = tid < N && tid >= from && Ab[tid * MAXN + j] != 0;
        const uint64_t m = __ballot(ok);
        if (lane == 0)
            cand[wave] = m ? wave * 64 + __builtin_ctzll(m) : (1 << 30);
        __syncthreads();
        const int pr = min(min(cand[0], cand[1]), min(cand[2], cand[3]));
        return pr;
    };
    auto swap_rows = [&](int a, int b) {
        if (a != b && tid < NW) {
            const uint32_t t = A[a * RW + tid];
            A[a * RW + tid] = A[b * RW + tid];
            A[b * RW + tid] = t;
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
            uint32_t a = A[j * RW + tid];
            const uint32_t pinv = IV[Ab[j * MAXN + j]];
            if (tid == (j >> 2))
                a = (a & ~(0xFFu << (8 * (j & 3)))) | (1u << (8 * (j & 3)));
            A[j * RW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        if (tid < N)
            fcol[tid] = tid == j ? 0 : Ab[tid * MAXN + j];
        __syncthreads();
        for (int it = tid; it < N * NW; it += 256) {
            const int i = it / NW, l = it - i * NW;
            const uint32_t f = fcol[i];
            if (f == 0)
                continue;
            uint32_t a = A[i * RW + l];
            if (l == (j >> 2))
                a &= ~(0xFFu << (8 * (j & 3)));
            a ^= prod4(T[f][0], T[f][1].x, A[j * RW + l]);
            A[i * RW + l] = a;
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
            Cinv[it] = Ab[i * MAXN + src[c]];
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
            const uint32_t pinv = IV[Ab[prow * MAXN + j]];
            const uint32_t a = A[prow * RW + tid];
            A[prow * RW + tid] = prod4(T[pinv][0], T[pinv][1].x, a);
        }
        __syncthreads();
        if (tid < N)
            fcol[tid] = tid > prow ? Ab[tid * MAXN + j] : 0;
        __syncthreads();
        for (int it = tid; it < N * NW; it += 256) {
            const int i = it / NW, l = it - i * NW;
            const uint32_t f = fcol[i];
            if (f == 0)
                continue;
            A[i * RW + l] ^= prod4(T[f][0], T[f][1].x, A[prow * RW + l]);
        }
        __syncthreads();
        prow++;
    }
    if (tid == 0 && rank_out)
        *rank_out = prow;
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

#define GF_ENC_DISPATCH(MACRO)                                                                                   \
    switch (v.D * 100 + v.KW) {                                                                                  \
    case 108: MACRO(1, 8); break;                                                                                \
    case 116: MACRO(1, 16); break;                                                                               \
    case 132: MACRO(1, 32); break;                                                                               \
    case 208: MACRO(2, 8); break;                                                                                \
    case 216: MACRO(2, 16); break;                                                                               \
    case 232: MACRO(2, 32); break;                                                                               \
    case 408: MACRO(4, 8); break;                                                                                \
    case 416: MACRO(4, 16); break;                                                                               \
    case 432: MACRO(4, 32); break;                                                                               \
    default: return hipErrorInvalidValue;                                                                        \
    }

hipError_t launch_encode(const Variant &v, const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s,
                         uint8_t *Y, uint64_t ld_y, uint64_t len, const uint32_t *ptab_field, const int *status,
                         int need, bool aligned, hipStream_t s)
{
    if (K <= 0 || len == 0)
        return hipSuccess;
    const uint64_t gx = (len + strip_bytes(v.D) - 1) / strip_bytes(v.D);
    const unsigned gy = (unsigned)((K + v.KW - 1) / v.KW);
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
#define GF_LAUNCH_ENC(DD, KK)                                                                                    \
    hipLaunchKernelGGL((k_encode<DD, KK>), dim3((unsigned)gx, gy), dim3(256), 0, s, C, K, N, S, ld_s, Y, ld_y,    \
                       len, pt, status, need, aligned ? 1 : 0)
    GF_ENC_DISPATCH(GF_LAUNCH_ENC)
#undef GF_LAUNCH_ENC
    return hipGetLastError();
}

hipError_t launch_encode_persistent(const Variant &v, const DevGen *gens, const DevTile *tiles, int ntiles,
                                    unsigned *counters, int grid, const uint32_t *ptab_field, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    const uint4 *pt = reinterpret_cast<const uint4 *>(ptab_field);
#define GF_LAUNCH_PERS(DD, KK)                                                                                   \
    hipLaunchKernelGGL((k_encode_persistent<DD, KK>), dim3(grid), dim3(256), 0, s, gens, tiles, ntiles, counters, \
                       pt)
    GF_ENC_DISPATCH(GF_LAUNCH_PERS)
#undef GF_LAUNCH_PERS
    return hipGetLastError();
}

int encode_blocks_per_cu(const Variant &v)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define GF_OCC(DD, KK)                                                                                           \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(                         \
                                                              &k_encode_persistent<DD, KK>),                      \
                                                     256, 0)
    switch (v.D * 100 + v.KW) {
    case 108: GF_OCC(1, 8); break;
    case 116: GF_OCC(1, 16); break;
    case 132: GF_OCC(1, 32); break;
    case 208: GF_OCC(2, 8); break;
    case 216: GF_OCC(2, 16); break;
    case 232: GF_OCC(2, 32); break;
    case 408: GF_OCC(4, 8); break;
    case 416: GF_OCC(4, 16); break;
    case 432: GF_OCC(4, 32); break;
    default: return 1;
    }
#undef GF_OCC
    if (e != hipSuccess || nb < 1)
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

}  // namespace gfnc
