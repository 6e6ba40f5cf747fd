// Device-side set-up of the batched calls that take their descriptors in
// device memory (include/gfnc.h: gf_encode_batched, gf_decode_batched).
//
// Encode: a plan holds the schedule (tiles and queues) of a list of shapes;
// at launch k_bind_gens reads the caller's descriptors, checks each against
// the shape the plan was built for and writes the launch's generation table,
// so one plan serves any buffers of those shapes without host work.
//
// Decode: no plan.  One workgroup (k_dec_schedule) reads the systems,
// checks them, sorts them into the elimination kernels' size classes and
// lays out the product's tiles in the persistent kernels' queues, all inside
// the caller's workspace; the eliminations and the product then run from
// those tables (Gauss-Jordan decoding, then S = C^-1 B: Sec. II, Eq. (1)).
#include "gf_internal.h"

namespace gfnc {

namespace {

// include/gfnc.h's gf_gen and gf_sys as the kernels read them.
struct ExtGen {
    const uint8_t *C;
    const uint8_t *S;
    uint8_t *Y;
    uint32_t K, N;
    uint64_t len, ld_s, ld_y;
};
struct ExtSys {
    const uint8_t *C;
    const uint8_t *B;
    uint8_t *S;
    uint32_t N, reserved;
    uint64_t len, ld_b, ld_s;
};

__device__ __forceinline__ uint32_t dev_row_align(const void *S, uint64_t ld_s, const void *Y, uint64_t ld_y)
{
    const uint64_t bits = (uint64_t)(uintptr_t)S | (uint64_t)(uintptr_t)Y | ld_s | ld_y;
    return bits % 16 == 0 ? 16u : bits % 8 == 0 ? 8u : bits % 4 == 0 ? 4u : 1u;
}

// Generation i of the launch: the plan's shape with the caller's pointers.  A
// descriptor whose shape differs from the plan's, whose pointers are missing,
// or whose rows are less aligned than the plan assumed is not run: its status
// points at a word that never equals `need` and the plan's error count grows.
__global__ __launch_bounds__(256) void k_bind_gens(const ExtGen *__restrict__ ext, const DevGen *__restrict__ shape,
                                                   DevGen *__restrict__ out, int count, unsigned *err,
                                                   const int *skip)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count)
        return;
    const ExtGen e = ext[i];
    DevGen g = shape[i];
    const bool work = g.K > 0 && g.len > 0;
    bool ok = e.K == g.K && e.N == g.N && e.len == g.len && (g.N <= 1 || e.ld_s == g.ld_s) &&
              (g.K <= 1 || e.ld_y == g.ld_y);
    ok = ok && (!work || (e.C && e.S && e.Y));
    ok = ok && (!work || dev_row_align(e.S, g.N > 1 ? e.ld_s : 0, e.Y, g.K > 1 ? e.ld_y : 0) >= g.align);
    g.C = e.C;
    g.S = e.S;
    g.Y = e.Y;
    if (!ok) {
        g.status = skip;   // *skip is 1, need is 0: every tile of it is skipped
        g.need = 0;
        atomicAdd(err, 1u);
    }
    out[i] = g;
}

constexpr int SCHED_THREADS = 1024;

// The decode schedule, built by one workgroup.  Valid systems (1 <= N <= 256,
// N^2 within the workspace's inverse slot, pitches >= len, pointers present,
// len <= 2^34) go to the size class of their elimination kernel (N <= 32, 64,
// 128, 256), get their inverse slot and a generation entry for the product
// S = C^-1 B (gated on rank N), and one tile per 16 coded rows in queue i % 8
// of the product kernel their rows allow (copies of 4-byte aligned source
// rows go straight to LDS; others take the byte-load kernel).  An invalid
// system gets rank -1 and nothing else.
__global__ __launch_bounds__(SCHED_THREADS) void k_dec_schedule(const ExtSys *__restrict__ sys, int count,
                                                                 DecSched w)
{
    __shared__ unsigned cls_n[4], cls_cur[4];
    __shared__ unsigned q_n[2][MF_QUEUES], q_cur[2][MF_QUEUES];
    const int tid = threadIdx.x;
    if (tid < 4)
        cls_n[tid] = 0;
    if (tid < 2 * MF_QUEUES)
        (&q_n[0][0])[tid] = 0;
    for (int i = tid; i < 2 * GF_QUEUE_CTR_WORDS; i += SCHED_THREADS)
        w.ctr[i] = 0;
    __syncthreads();

    auto classify = [&](int i, int &c, int &sel, int &nt) -> bool {
        const ExtSys s = sys[i];
        const uint64_t N = s.N;
        bool ok = N >= 1 && N <= 256 && N * N <= w.slot && s.C && s.len <= (1ull << 34);
        ok = ok && (s.len == 0 || (s.B && s.S && (N <= 1 || (s.ld_b >= s.len && s.ld_s >= s.len))));
        c = N <= 32 ? 0 : N <= 64 ? 1 : N <= 128 ? 2 : 3;
        sel = (((uintptr_t)s.B | (N > 1 ? s.ld_b : 0)) % 4 == 0) ? 0 : 1;
        nt = s.len > 0 ? (int)((N + MF_ROWS - 1) / MF_ROWS) : 0;
        return ok;
    };

    for (int i = tid; i < count; i += SCHED_THREADS) {
        int c, sel, nt;
        if (classify(i, c, sel, nt)) {
            atomicAdd(&cls_n[c], 1u);
            if (nt)
                atomicAdd(&q_n[sel][i % MF_QUEUES], (unsigned)nt);
        }
    }
    __syncthreads();
    if (tid == 0) {
        for (int c = 0; c < 4; c++) {
            w.cls_count[c] = cls_n[c];
            cls_cur[c] = 0;
        }
        for (int sel = 0; sel < 2; sel++) {
            unsigned acc = 0;
            for (int q = 0; q < MF_QUEUES; q++) {
                w.bounds[sel * (MF_QUEUES + 1) + q] = acc;
                q_cur[sel][q] = acc;
                acc += q_n[sel][q];
            }
            w.bounds[sel * (MF_QUEUES + 1) + MF_QUEUES] = acc;
        }
    }
    __syncthreads();

    for (int i = tid; i < count; i += SCHED_THREADS) {
        int c, sel, nt;
        const bool ok = classify(i, c, sel, nt);
        int *rank = w.rank + i;
        if (!ok) {
            *rank = -1;
            continue;
        }
        const ExtSys s = sys[i];
        uint8_t *cinv = w.inv + (uint64_t)i * w.slot;
        const unsigned at = atomicAdd(&cls_cur[c], 1u);
        w.lists[(uint64_t)c * count + at] = DevSys{s.C, cinv, rank, s.N, 0};
        w.gens[i] = DevGen{cinv, s.B, s.S, s.len, s.ld_b, s.ld_s, s.N, s.N, rank, (int)s.N,
                           dev_row_align(s.B, s.N > 1 ? s.ld_b : 0, s.S, s.N > 1 ? s.ld_s : 0)};
        if (nt) {
            const unsigned t0 = atomicAdd(&q_cur[sel][i % MF_QUEUES], (unsigned)nt);
            DevTile *tl = w.tiles + (uint64_t)sel * w.tile_cap;
            for (int k = 0; k < nt; k++)
                tl[t0 + k] = DevTile{(uint32_t)i, (uint16_t)(k * MF_ROWS), 0, 0};
        }
    }
}

}  // namespace

hipError_t launch_bind_gens(const void *d_ext, const DevGen *shape, DevGen *out, int count, unsigned *err,
                            const int *skip, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_bind_gens, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       static_cast<const ExtGen *>(d_ext), shape, out, count, err, skip);
    return hipGetLastError();
}

hipError_t launch_dec_schedule(const void *d_sys, int count, const DecSched &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_schedule, dim3(1), dim3(SCHED_THREADS), 0, s, static_cast<const ExtSys *>(d_sys),
                       count, w);
    return hipGetLastError();
}

}  // namespace gfnc
