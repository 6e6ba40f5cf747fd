// The C ABI (include/gfnc.h): argument validation, device tables, plans for
// the batched launches, and HIP-graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <numeric>
#include <cstring>
#include <vector>

#include "../../include/gfnc.h"
#include "gf_internal.h"

using namespace gfnc;

namespace gfnc {

// Largest of 16, 8, 4 (else 1) that divides every row start: the widest
// vector access the rows allow.
uint32_t row_align(const void *S, uint64_t ld_s, const void *Y, uint64_t ld_y)
{
    const uint64_t bits = (uint64_t)(uintptr_t)S | (uint64_t)(uintptr_t)Y | ld_s | ld_y;
    for (uint32_t a : {16u, 8u, 4u})
        if (bits % a == 0)
            return a;
    return 1;
}

}  // namespace gfnc

namespace {

constexpr int kMaxDevices = 64;

// Scratch memory of gf_decode_noalloc: the inverse of up to GF_MAX_N x
// GF_MAX_N, then the rank.  Every device holds its own copy until the process
// ends.  In host code this name is only a handle for hipGetSymbolAddress; the
// device address found at set-up (DevState::scratch) is what kernels get.
constexpr size_t kScratchInverse = (size_t)GF_MAX_N * GF_MAX_N;
constexpr size_t kScratchBytes = kScratchInverse + 256;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DevState {
    bool ready = false;
    DevTables t{nullptr, nullptr, nullptr};
    int cus = 0;
    uint8_t *scratch = nullptr;   // device address of `scratch` on this device
};

std::mutex g_mu;
DevState g_dev[kMaxDevices];

int current_state(DevState **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return GF_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[dev];
    if (!d.ready) {
        const HostTables &h = host_tables();
        void *pt = nullptr, *iv = nullptr, *rw = nullptr;
        // the product tables, then those of every element's inverse (the same layout)
        std::vector<uint32_t> tabs(2 * sizeof h.ptab / sizeof(uint32_t));
        std::memcpy(tabs.data(), h.ptab, sizeof h.ptab);
        for (int f = 0; f < 4; f++)
            for (int c = 0; c < 256; c++)
                std::memcpy(&tabs[((size_t)(4 + f) * 256 + c) * 8], h.ptab[f][h.inv[f][c]], 8 * sizeof(uint32_t));
        if (hipMalloc(&pt, 2 * sizeof h.ptab) != hipSuccess)
            return GF_EDEVICE;
        if (hipMalloc(&iv, sizeof h.inv) != hipSuccess || hipMalloc(&rw, sizeof h.rows) != hipSuccess) {
            (void)hipFree(pt);
            (void)hipFree(iv);
            return GF_EDEVICE;
        }
        if (hipMemcpy(pt, tabs.data(), 2 * sizeof h.ptab, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(iv, h.inv, sizeof h.inv, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(rw, h.rows, sizeof h.rows, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(pt);
            (void)hipFree(iv);
            (void)hipFree(rw);
            return GF_EDEVICE;
        }
        // this device's copy of the scratch array (the device is current here)
        void *sp = nullptr;
        if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
            (void)hipFree(pt);
            (void)hipFree(iv);
            (void)hipFree(rw);
            return GF_EDEVICE;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        d.scratch = static_cast<uint8_t *>(sp);
        d.t.ptab = static_cast<uint32_t *>(pt);
        d.t.inv = static_cast<uint8_t *>(iv);
        d.t.rows = static_cast<uint8_t *>(rw);
        d.cus = cus;
        d.ready = true;
    }
    *out = &d;
    return GF_OK;
}

// The state of the current device only if gf_init (or any other call) has
// already set it up: GF_ENOTINIT otherwise.  Allocates nothing.
int ready_state(DevState **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return GF_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev[dev].ready)
        return GF_ENOTINIT;
    *out = &g_dev[dev];
    return GF_OK;
}

bool valid_field(int f) { return f == 1 || f == 2 || f == 4 || f == 8; }

const uint32_t *field_ptab(const DevState *d, int field)
{
    return d->t.ptab + (size_t)field_index(field) * 256 * 8;
}
const uint32_t *field_ptab_inv(const DevState *d, int field)
{
    return d->t.ptab + (size_t)(4 + field_index(field)) * 256 * 8;
}
const uint8_t *field_inv(const DevState *d, int field) { return d->t.inv + (size_t)field_index(field) * 256; }
const uint8_t *field_rows(const DevState *d, int field) { return d->t.rows + (size_t)field_index(field) * 256 * 8; }

int dev_err(hipError_t e) { return e == hipSuccess ? GF_OK : GF_EDEVICE; }

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    if (na == 0 || nb == 0)
        return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

size_t envelope(size_t rows, size_t ld, size_t len) { return rows == 0 || len == 0 ? 0 : (rows - 1) * ld + len; }

// Byte span of `rows` rows `ld` apart, `len` bytes each, starting at p (0 when
// empty); false when the span or its end address does not fit in 64 bits, so
// the overlap checks never see a wrapped size.
bool span_of(const void *p, size_t rows, size_t ld, size_t len, size_t *out)
{
    size_t n = 0;
    if (rows > 0 && len > 0) {
        if (rows > 1 && ld > (SIZE_MAX - len) / (rows - 1))
            return false;
        n = (rows - 1) * ld + len;
    }
    if (n > UINTPTR_MAX - (uintptr_t)p)
        return false;
    *out = n;
    return true;
}

// Stand-in addresses for validating a shape-only descriptor: 16-byte aligned,
// 2^60 bytes apart so that no legal shape makes them overlap; never used.
const uint8_t *const kShapeC = reinterpret_cast<const uint8_t *>(uintptr_t(1) << 60);
const uint8_t *const kShapeS = reinterpret_cast<const uint8_t *>(uintptr_t(2) << 60);
uint8_t *const kShapeY = reinterpret_cast<uint8_t *>(uintptr_t(3) << 60);

struct Single {
    int D;
    int nsplit;
};

// Schedule of a single-generation launch.  Lane width: padded payload work,
// inflated for narrow lanes (more table reads per byte).  When the tiles do
// not fill the GPU (2 waves on each of its SIMDs), the sources are split into
// slices whose partial sums are XORed into the output with atomics, provided
// the rows are 4-byte aligned and every slice keeps at least 8 sources.
Single pick_single(int K, int N, uint64_t len, uint32_t align, int cus)
{
    Single best{1, 1};
    double best_cost = 1e300;
    const double fill = (double)cus * 8.0;
    const bool can_split = align >= 4 && len >= 4;
    for (int D : {4, 2, 1}) {
        const uint64_t s = wave_strip(D);
        const double strips = (double)((len + s - 1) / s);
        const double tiles = strips * (double)((K + ENC_ROWS - 1) / ENC_ROWS);
        int split = 1;
        if (can_split && tiles < fill)
            split = std::max(1, std::min((int)std::ceil(fill / tiles), N / 8));
        const double par = std::min(1.0, tiles * split / fill);
        const double cost = strips * (double)s * (1.0 + 0.15 / D) * (1.0 + 0.02 * split) / par;
        if (cost < best_cost) {
            best_cost = cost;
            best = Single{D, split};
        }
    }
    return best;
}

}  // namespace

// =========================================================================

struct gf_plan {
    int kind = 0;     // 0 encode, 1 decode, 2 recode (payloads here, headers in `head`)
    int field = 8;
    int dev = 0;
    int count = 0;
    int fixed_D = 0;   // 0: lane width chosen per tile
    int form = 1;      // 1 table (VALU byte-select), 2 bit-matrix on the matrix cores, 3 bit-plane (VALU)
    bool src_aligned4 = false;   // every generation's source rows start 4-byte aligned
    std::vector<TuneChoice> trials;     // the autotuner's timed candidates
    bool tuned_from_cache = false;
    int grid = 0;
    bool direct = false;   // forms 1 and 3: a workgroup per four wave tiles, not persistent
    int ntiles = 0;
    DevGen *d_gens = nullptr;       // the generations as described when the plan was made
    DevGen *d_bound = nullptr;      // the same shapes with the pointers of gf_encode_batched's descriptors
    unsigned *d_err = nullptr;      // [0] descriptors refused by that call, [1] = 1 (status of a refused one)
    bool shape_only = false;        // made from shapes alone (no pointers to run on)
    bool small_ok = false;          // every generation has K, N <= STREAM_MAX and 16-byte aligned rows (forms 4 and 5 apply)
    int small_max = 0;              // the largest K or N of the batch
    DevTile *d_tiles = nullptr;
    unsigned *d_runs = nullptr;     // first tile of each run, then the queue bounds
    unsigned *d_bounds = nullptr;   // inside d_runs
    unsigned *d_ctr = nullptr;
    // decode
    DevSys *d_sys = nullptr;
    uint8_t *d_cinv = nullptr;
    int *d_rank = nullptr;
    int class_begin[4] = {0, 0, 0, 0};
    int class_count[4] = {0, 0, 0, 0};
    std::vector<int> sys_order;       // plan position -> caller's index
    // graph replay
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int *graph_rank = nullptr;
    // host copy of the descriptors (for gf_encode_each-style diagnostics)
    std::vector<gf_gen> gens;
    // recode: the encode plan of the coefficient headers, launched first
    gf_plan *head = nullptr;
    // decode: the product S = Cinv B of each size class (an encode plan each),
    // and streams and events that let the size classes' work overlap
    gf_plan *prod[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_done[3] = {nullptr, nullptr, nullptr};
};

int gfnc::gfnc_field_tables(int field, const uint32_t **ptab, const uint8_t **inv)
{
    if (!valid_field(field))
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    *ptab = field_ptab(d, field);
    *inv = field_inv(d, field);
    return GF_OK;
}

const uint8_t *gfnc::gfnc_field_rows(int field)
{
    DevState *d;
    if (!valid_field(field) || current_state(&d))
        return nullptr;
    return field_rows(d, field);
}

extern "C" {

int gf_init(void)
{
    DevState *d;
    return current_state(&d);
}

const char *gf_strerror(int code)
{
    switch (code) {
    case GF_OK: return "success";
    case GF_EINVAL: return "invalid argument";
    case GF_ENOTINIT: return "library not initialised";
    case GF_EDEVICE: return "HIP runtime error";
    case GF_ESINGULAR: return "coefficient matrix is singular";
    case GF_ENOMEM: return "out of memory";
    case GF_ERANGE: return "size above the supported maximum";
    case GF_ECANCELED: return "request cancelled";
    default: return "unknown error";
    }
}

static int region_common(int mode, int field, uint8_t *y, const uint8_t *x, int c, size_t len, void *stream)
{
    if (!valid_field(field) || c < 0 || c >= (1 << field))
        return GF_EINVAL;
    if (len == 0)
        return GF_OK;
    size_t ny, nx;
    if (!y || !x || !span_of(y, 1, 0, len, &ny) || !span_of(x, 1, 0, len, &nx))
        return GF_EINVAL;
    if (y != x && overlap(y, ny, x, nx))
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    if (mode == 0 && c == 0)
        return GF_OK;
    const uint32_t *t = host_tables().ptab[field_index(field)][c];
    return dev_err(launch_region(mode, y, x, len, t, (hipStream_t)stream));
}

int gf_region_madd(int field, uint8_t *y, const uint8_t *x, int c, size_t len, void *stream)
{
    return region_common(0, field, y, x, c, len, stream);
}

int gf_region_mul(int field, uint8_t *y, const uint8_t *x, int c, size_t len, void *stream)
{
    return region_common(1, field, y, x, c, len, stream);
}

int gf_region_madd_batched(int field, const gf_region *d_regions, int count, size_t max_len, void *stream)
{
    if (!valid_field(field) || count < 0)
        return GF_EINVAL;
    if (count == 0 || max_len == 0)
        return GF_OK;
    if (!d_regions)
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    return dev_err(launch_region_batched(d_regions, count, max_len, field_ptab(d, field), 1 << field,
                                         (hipStream_t)stream));
}

static int check_encode_args(int field, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s,
                             const uint8_t *Y, size_t ld_y, size_t len)
{
    if (!valid_field(field) || K < 0 || N < 1)
        return GF_EINVAL;
    if (N > GF_MAX_N)
        return GF_ERANGE;
    if (K == 0 || len == 0)
        return GF_OK;
    if (!C || !S || !Y)
        return GF_EINVAL;
    if ((N > 1 && ld_s < len) || (K > 1 && ld_y < len))
        return GF_EINVAL;
    size_t ey, es, ec;
    if (!span_of(Y, K, ld_y, len, &ey) || !span_of(S, N, ld_s, len, &es) || !span_of(C, K, N, N, &ec))
        return GF_EINVAL;
    if (overlap(Y, ey, S, es) || overlap(Y, ey, C, ec))
        return GF_EINVAL;
    return GF_OK;
}

static int encode_impl(int field, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s, uint8_t *Y,
                       size_t ld_y, size_t len, const gf_tuning *tune, const int *status, int need, void *stream)
{
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    const uint32_t al = row_align(S, N > 1 ? ld_s : 0, Y, K > 1 ? ld_y : 0);
    if (!status && !(tune && tune->bytes_per_lane) && small_ok(K, N, len, al))
        return dev_err(launch_small(C, K, N, S, ld_s, Y, ld_y, len, field_ptab(d, field), field_ptab_inv(d, field),
                                    field_inv(d, field), nullptr,
                                    false, (hipStream_t)stream));
    Single sc = pick_single(K, N, len, al, d->cus);
    if (tune && tune->bytes_per_lane) {
        if (tune->bytes_per_lane != 4 && tune->bytes_per_lane != 8 && tune->bytes_per_lane != 16)
            return GF_EINVAL;
        sc.D = tune->bytes_per_lane / 4;
    }
    return dev_err(launch_encode(sc.D, sc.nsplit, C, K, N, S, ld_s, Y, ld_y, len, field_ptab(d, field), status, need,
                                 al >= 4u * (uint32_t)sc.D, (hipStream_t)stream));
}

int gf_encode(int field, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s, uint8_t *Y, size_t ld_y,
              size_t len, void *stream)
{
    int rc = check_encode_args(field, C, K, N, S, ld_s, Y, ld_y, len);
    if (rc || K == 0 || len == 0)
        return rc;
    return encode_impl(field, C, K, N, S, ld_s, Y, ld_y, len, nullptr, nullptr, 0, stream);
}

int gf_encode_each(int field, const gf_gen *gens, int count, const gf_tuning *tune, void *stream)
{
    if (count < 0 || (count > 0 && !gens) || !valid_field(field))
        return GF_EINVAL;
    for (int i = 0; i < count; i++) {
        const gf_gen &g = gens[i];
        int rc = check_encode_args(field, g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len);
        if (rc)
            return rc;
    }
    for (int i = 0; i < count; i++) {
        const gf_gen &g = gens[i];
        if (g.K == 0 || g.len == 0)
            continue;
        int rc = encode_impl(field, g.C, (int)g.K, (int)g.N, g.S, g.ld_s, g.Y, g.ld_y, g.len, tune, nullptr, 0,
                             stream);
        if (rc)
            return rc;
    }
    return GF_OK;
}

// Bytes of one inverse of up to max_N x max_N, rounded to 256.
static size_t inverse_bytes(int max_N) { return (((size_t)max_N * max_N + 255) / 256) * 256; }

static size_t r256(size_t x) { return (x + 255) / 256 * 256; }

// Where gf_decode_batched keeps its tables in the workspace (byte offsets),
// before the inverses; `fixed` is their total.
struct DecWsLayout {
    size_t hdr, ctr, lists, gens, tiles, rank, fixed;
    uint64_t tile_cap;
};

static DecWsLayout dec_ws_layout(size_t count)
{
    DecWsLayout L;
    size_t off = 0;
    L.hdr = off;     // class counts [4], queue bounds [2][MF_QUEUES + 1]
    off += 256;
    L.ctr = off;
    off += r256(2 * GF_QUEUE_CTR_WORDS * sizeof(unsigned));
    L.lists = off;
    off += r256(4 * count * sizeof(DevSys));
    L.gens = off;
    off += r256(count * sizeof(DevGen));
    L.tile_cap = (uint64_t)count * ((GF_MAX_N + MF_ROWS - 1) / MF_ROWS);
    L.tiles = off;
    off += r256(2 * L.tile_cap * sizeof(DevTile));
    L.rank = off;
    off += r256(count * sizeof(int));
    L.fixed = off;
    return L;
}

size_t gf_decode_workspace(int field, int max_N, int count)
{
    if (!valid_field(field) || max_N < 1 || max_N > GF_MAX_N || count < 1)
        return 0;
    return dec_ws_layout((size_t)count).fixed + (size_t)count * inverse_bytes(max_N);
}

int gf_invert(int field, const uint8_t *C, int N, uint8_t *Cinv, int *d_rank, void *stream)
{
    if (!valid_field(field) || N < 1 || !C || !Cinv)
        return GF_EINVAL;
    if (N > GF_MAX_N)
        return GF_ERANGE;
    size_t nc, ni;
    if (!span_of(C, N, N, N, &nc) || !span_of(Cinv, N, N, N, &ni) || overlap(C, nc, Cinv, ni))
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    return dev_err(launch_invert(nullptr, 0, C, N, Cinv, d_rank, field_ptab(d, field), field_inv(d, field),
                                 (hipStream_t)stream));
}

// Checks of a decode's matrix and rows (the workspace aside).
static int check_decode_args(int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, const uint8_t *S,
                             size_t ld_s, size_t len, size_t *es, size_t *eb, size_t *ec)
{
    if (!valid_field(field) || N < 1)
        return GF_EINVAL;
    if (N > GF_MAX_N)
        return GF_ERANGE;
    if (!C)
        return GF_EINVAL;
    if (len > 0 && (!B || !S || (N > 1 && (ld_b < len || ld_s < len))))
        return GF_EINVAL;
    if (!span_of(S, N, ld_s, len, es) || !span_of(B, N, ld_b, len, eb) || !span_of(C, N, N, N, ec))
        return GF_EINVAL;
    if (overlap(S, *es, B, *eb) || overlap(S, *es, C, *ec))
        return GF_EINVAL;
    return GF_OK;
}

// S = C^-1 B with the inverse written to `cinv` (N^2 bytes) and the rank to
// `rank` (both device memory the caller of this function provides).
static int decode_impl(DevState *d, int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, uint8_t *S,
                       size_t ld_s, size_t len, uint8_t *cinv, int *rank, void *stream)
{
    if (small_ok(N, N, len, row_align(B, N > 1 ? ld_b : 0, S, N > 1 ? ld_s : 0)))
        return dev_err(launch_small(C, N, N, B, ld_b, S, ld_s, len, field_ptab(d, field), field_ptab_inv(d, field),
                                    field_inv(d, field), rank,
                                    true, (hipStream_t)stream));
    hipError_t e = launch_invert(nullptr, 0, C, N, cinv, rank, field_ptab(d, field), field_inv(d, field),
                                 (hipStream_t)stream);
    if (e != hipSuccess)
        return GF_EDEVICE;
    if (len == 0)
        return GF_OK;
    return encode_impl(field, cinv, N, N, B, ld_b, S, ld_s, len, nullptr, rank, N, stream);
}

int gf_decode(int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, uint8_t *S, size_t ld_s,
              size_t len, void *ws, size_t ws_bytes, int *d_rank, void *stream)
{
    size_t es, eb, ec, ew;
    int rc = check_decode_args(field, C, B, ld_b, N, S, ld_s, len, &es, &eb, &ec);
    if (rc)
        return rc;
    if (!ws || ws_bytes < gf_decode_workspace(field, N, 1) || !span_of(ws, 1, 0, ws_bytes, &ew))
        return GF_EINVAL;
    if (overlap(S, es, ws, ew) || overlap(ws, ew, C, ec) || overlap(ws, ew, B, eb))
        return GF_EINVAL;
    DevState *d;
    if ((rc = current_state(&d)))
        return rc;
    uint8_t *cinv = static_cast<uint8_t *>(ws);
    int *rank = d_rank ? d_rank : reinterpret_cast<int *>(cinv + inverse_bytes(N));
    return decode_impl(d, field, C, B, ld_b, N, S, ld_s, len, cinv, rank, stream);
}

int gf_decode_noalloc(int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, uint8_t *S, size_t ld_s,
                      size_t len, int *d_rank, void *stream)
{
    size_t es, eb, ec;
    int rc = check_decode_args(field, C, B, ld_b, N, S, ld_s, len, &es, &eb, &ec);
    if (rc)
        return rc;
    static_assert((size_t)GF_MAX_N * GF_MAX_N <= kScratchInverse, "scratch holds the largest inverse");
    DevState *d;
    if ((rc = ready_state(&d)))
        return rc;
    uint8_t *cinv = d->scratch;
    int *rank = d_rank ? d_rank : reinterpret_cast<int *>(d->scratch + kScratchInverse);
    return decode_impl(d, field, C, B, ld_b, N, S, ld_s, len, cinv, rank, stream);
}

// ------------------------------------------------------------------ plans

static void plan_free_device(gf_plan *p)
{
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->cap)
        (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->d_gens);
    (void)hipFree(p->d_bound);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_tiles);
    (void)hipFree(p->d_runs);
    (void)hipFree(p->d_ctr);
    (void)hipFree(p->d_sys);
    (void)hipFree(p->d_cinv);
    (void)hipFree(p->d_rank);
    if (p->head) {
        plan_free_device(p->head);
        delete p->head;
        p->head = nullptr;
    }
    for (gf_plan *&q : p->prod) {
        if (q) {
            plan_free_device(q);
            delete q;
            q = nullptr;
        }
    }
    for (int i = 0; i < 3; i++) {
        if (p->aux[i])
            (void)hipStreamDestroy(p->aux[i]);
        if (p->ev_done[i])
            (void)hipEventDestroy(p->ev_done[i]);
    }
    if (p->ev_fork)
        (void)hipEventDestroy(p->ev_fork);
}

}  // extern "C"

template <class T>
static int upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty())
        return GF_OK;
    if (hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)) != hipSuccess)
        return GF_ENOMEM;
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return GF_EDEVICE;
    return GF_OK;
}

namespace gfnc {

// Wave tiles of one generation: per block of ENC_ROWS coded rows, strips of
// 256*D bytes (D = 4 while more than 512 bytes remain; a packet's last partial
// strip uses the narrowest lane width that covers it, so at most a few lanes
// idle).  `fixed_D` forces one width for every strip.  Consecutive strips of
// one width share a tile while the tile's byte products stay below 2^18
// (short generations: fewer claims and descriptor loads per byte).
static void gen_tiles(uint32_t gi, const DevGen &x, int fixed_D, std::vector<std::pair<DevTile, double>> &out)
{
    if (x.K == 0 || x.len == 0)
        return;
    auto width = [&](uint64_t rest) {
        return fixed_D ? fixed_D : rest > wave_strip(2) ? 4 : rest > wave_strip(1) ? 2 : 1;
    };
    for (uint32_t k0 = 0; k0 < x.K; k0 += ENC_ROWS) {
        const double rows = (double)std::min<uint32_t>(ENC_ROWS, x.K - k0);
        uint64_t p0 = 0;
        while (p0 < x.len) {
            const int D = width(x.len - p0);
            const double per = (double)x.N * rows * (double)wave_strip(D);
            int strips = 1;
            while (strips < 256 && per * (strips + 1) <= 262144.0) {
                const uint64_t next = p0 + (uint64_t)strips * wave_strip(D);
                if (next >= x.len || width(x.len - next) != D)
                    break;
                strips++;
            }
            out.push_back({DevTile{gi, (uint16_t)k0, (uint16_t)(D | ((strips - 1) << 8)), p0}, per * strips});
            p0 += (uint64_t)strips * wave_strip(D);
        }
    }
}

// Work queues from the tiles of every generation (each generation's tiles
// contiguous in `tiles`, with a cost each): generations go to the MF_QUEUES
// queues largest first, each to the least loaded one; inside a queue the
// tiles run longest first (LPT order; ties keep a generation's tiles
// together), and consecutive tiles are grouped into runs of cost >= run_cost.
static void build_queues(const std::vector<std::pair<DevTile, double>> &tiles, double run_cost, TileQueues &q)
{
    struct Span {
        size_t first, count;
        double cost;
    };
    std::vector<Span> gens;
    for (size_t i = 0; i < tiles.size(); i++) {
        if (gens.empty() || tiles[i].first.gen != tiles[gens.back().first].first.gen)
            gens.push_back({i, 0, 0.0});
        gens.back().count++;
        gens.back().cost += tiles[i].second;
    }
    std::stable_sort(gens.begin(), gens.end(), [](const Span &a, const Span &b) { return a.cost > b.cost; });
    std::vector<size_t> member[MF_QUEUES];
    double load[MF_QUEUES] = {};
    for (const Span &x : gens) {
        int best = 0;
        for (int i = 1; i < MF_QUEUES; i++)
            if (load[i] < load[best])
                best = i;
        for (size_t k = 0; k < x.count; k++)
            member[best].push_back(x.first + k);
        load[best] += x.cost;
    }
    q.tiles.clear();
    q.runs.clear();
    for (int i = 0; i < MF_QUEUES; i++) {
        q.bounds[i] = (unsigned)q.runs.size();
        std::stable_sort(member[i].begin(), member[i].end(),
                         [&](size_t a, size_t b) { return tiles[a].second > tiles[b].second; });
        double acc = 0;
        for (size_t k : member[i]) {
            if (acc == 0)
                q.runs.push_back((unsigned)q.tiles.size());
            q.tiles.push_back(tiles[k].first);
            acc += tiles[k].second;
            if (acc >= run_cost)
                acc = 0;
        }
    }
    q.bounds[MF_QUEUES] = (unsigned)q.runs.size();
    q.runs.push_back((unsigned)q.tiles.size());
}

// Table form; a tile's cost is its byte products, and runs hold >= 2^18.
void build_tiles(const DevGen *g, size_t n, int fixed_D, TileQueues &q)
{
    std::vector<std::pair<DevTile, double>> tiles;
    for (size_t i = 0; i < n; i++)
        gen_tiles((uint32_t)i, g[i], fixed_D, tiles);
    build_queues(tiles, 262144.0, q);
}

// Bit-matrix form: one tile per MF_ROWS coded rows, cost ~ source groups x
// (strips + 1); runs hold >= 48.
void build_tiles_mfma(const DevGen *g, size_t n, TileQueues &q)
{
    std::vector<std::pair<DevTile, double>> tiles;
    for (size_t i = 0; i < n; i++) {
        const DevGen &x = g[i];
        if (x.K == 0 || x.len == 0)
            continue;
        const double strips = (double)((x.len + MF_STRIP - 1) / MF_STRIP);
        for (uint32_t k0 = 0; k0 < x.K; k0 += MF_ROWS)
            tiles.push_back({DevTile{(uint32_t)i, (uint16_t)k0, 0, 0}, (double)((x.N + 7) / 8) * (strips + 1.0)});
    }
    build_queues(tiles, 48.0, q);
}

// Small-generation streaming form: per generation, tiles of up to
// STREAM_STRIPS strips of 1 KiB over its whole length (every coded row in one
// tile); a tile's cost is the bytes it moves, and runs hold >= 2^18 of it.
void build_tiles_stream(const DevGen *g, size_t n, TileQueues &q)
{
    std::vector<std::pair<DevTile, double>> tiles;
    for (size_t i = 0; i < n; i++) {
        const DevGen &x = g[i];
        if (x.K == 0 || x.len == 0)
            continue;
        const uint64_t nstrips = (x.len + 1023) / 1024;
        for (uint64_t s0 = 0; s0 < nstrips; s0 += STREAM_STRIPS) {
            const uint64_t ns = std::min<uint64_t>(STREAM_STRIPS, nstrips - s0);
            const double bytes = (double)std::min<uint64_t>(x.len - s0 * 1024, ns * 1024);
            tiles.push_back({DevTile{(uint32_t)i, 0, (uint16_t)(4 | ((ns - 1) << 8)), s0 * 1024},
                             bytes * (double)(x.N + x.K)});
        }
    }
    build_queues(tiles, 262144.0, q);
}

// Chunked streaming form: each generation's strips of 1 KiB in runs of equal
// length (at most `burst` strips), in generation order.
void build_tiles_chunks(const DevGen *g, size_t n, int burst, std::vector<DevTile> &tiles)
{
    for (size_t i = 0; i < n; i++) {
        const DevGen &x = g[i];
        if (x.K == 0 || x.len == 0)
            continue;
        const uint64_t ns = (x.len + 1023) / 1024;
        const uint64_t runs = (ns + burst - 1) / burst;
        for (uint64_t r = 0; r < runs; r++) {
            const uint64_t s0 = r * ns / runs, s1 = (r + 1) * ns / runs;
            tiles.push_back(DevTile{(uint32_t)i, 0, (uint16_t)(4 | ((s1 - s0 - 1) << 8)), s0 * 1024});
        }
    }
}

}  // namespace gfnc

// One launch of the plan's persistent kernel over the generation table
// `gens` (the plan's own, or the one gf_encode_batched bound).
static int launch_schedule(gf_plan *p, DevState *d, hipStream_t s, const DevGen *gens = nullptr)
{
    const int f = p->field;
    if (!gens)
        gens = p->d_gens;
    hipError_t e;
    if (p->form == 2)
        e = launch_encode_mfma(gens, p->d_tiles, p->d_runs, p->d_bounds, p->ntiles, p->d_ctr, p->grid,
                               field_rows(d, f), p->src_aligned4, s);
    else if (p->form == 3)
        e = launch_encode_planes(f, gens, p->d_tiles, p->d_runs, p->d_bounds, p->ntiles, p->d_ctr, p->grid, s,
                                 p->direct);
    else if (p->form == 4)
        e = launch_encode_stream(p->small_max, gens, p->d_tiles, p->d_runs, p->d_bounds, p->ntiles, p->d_ctr,
                                 p->grid, field_ptab(d, f), s);
    else if (p->form == 5)
        e = launch_encode_chunks(p->small_max, gens, p->d_tiles, p->ntiles, field_ptab(d, f), s);
    else
        e = launch_encode_persistent(gens, p->d_tiles, p->d_runs, p->d_bounds, p->ntiles, p->d_ctr, p->grid,
                                     field_ptab(d, f), s, p->direct);
    return dev_err(e);
}

// Tile list, grid and device copies for one form.
// Workgroups of the full persistent grid of a form (as many as fit at once).
static int full_grid(const gf_plan *p, const DevState *d, int form)
{
    return d->cus * (form == 2   ? encode_mfma_blocks_per_cu(p->src_aligned4)
                     : form == 3 ? encode_planes_blocks_per_cu(p->field)
                     : form == 4 ? encode_stream_blocks_per_cu(p->small_max)
                                 : encode_blocks_per_cu());
}

// grid_pct: share of the full grid (100 unless the tuner tries less); 0 for
// forms 1 and 3: not persistent, a workgroup per four wave tiles.
static int make_schedule(gf_plan *p, DevState *d, const std::vector<DevGen> &g, int form, const gf_tuning *tune,
                         int grid_pct = 100)
{
    TileQueues tq;
    if (form == 2)
        build_tiles_mfma(g.data(), g.size(), tq);
    else if (form == 4)
        build_tiles_stream(g.data(), g.size(), tq);
    else if (form == 5)
        build_tiles_chunks(g.data(), g.size(), encode_chunks_strips(p->small_max), tq.tiles);
    else
        build_tiles(g.data(), g.size(), p->fixed_D, tq);
    (void)hipFree(p->d_tiles);
    (void)hipFree(p->d_runs);
    p->d_tiles = nullptr;
    p->d_runs = p->d_bounds = nullptr;
    p->form = form;
    p->ntiles = (int)tq.tiles.size();
    std::vector<unsigned> rb = tq.runs;   // runs, then the queue bounds
    rb.insert(rb.end(), tq.bounds, tq.bounds + MF_QUEUES + 1);
    int rc = upload(&p->d_tiles, tq.tiles);
    if (!rc)
        rc = upload(&p->d_runs, rb);
    if (rc)
        return rc;
    p->d_bounds = p->d_runs + tq.runs.size();
    int grid = std::max(1, full_grid(p, d, form) * std::max(grid_pct, 1) / 100);
    if (tune && tune->grid_blocks > 0)
        grid = tune->grid_blocks;
    const int per_block = form == 2 ? 1 : 4;
    p->grid = std::max(1, std::min(grid, std::max(1, (p->ntiles + per_block - 1) / per_block)));
    p->direct = (form == 1 || form == 3) && (grid_pct == 0 || (tune && tune->grid_blocks == -1));
    if (form == 5 || p->direct)   // not persistent: a workgroup per four tiles
        p->grid = std::max(1, (p->ntiles + 3) / 4);
    return GF_OK;
}

// Median milliseconds of `reps` launches of the current schedule over the
// generation table `gens`, after one untimed launch; -1 on an error.
static double time_schedule(gf_plan *p, DevState *d, const DevGen *gens, int reps = 3)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<double> ms;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        launch_schedule(p, d, p->cap, gens) == GF_OK) {
        for (int r = 0; r < reps; r++) {
            float f = 0;
            if (hipEventRecord(e0, p->cap) != hipSuccess || launch_schedule(p, d, p->cap, gens) != GF_OK ||
                hipEventRecord(e1, p->cap) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&f, e0, e1) != hipSuccess)
                break;
            ms.push_back(f);
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if ((int)ms.size() < reps)
        return -1;
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// Scratch memory the tuning trials run on, so that they never write the
// caller's outputs (and a plan of shapes has inputs to read): every trial's
// generation table points its outputs, and for a plan of shapes its inputs,
// into these buffers at the same offsets the rows have relative to each other.
struct TrialBuffers {
    uint8_t *y = nullptr, *s = nullptr, *c = nullptr;
    ~TrialBuffers()
    {
        (void)hipFree(y);
        (void)hipFree(s);
        (void)hipFree(c);
    }
};

static int trial_table(gf_plan *p, const std::vector<DevGen> &g, TrialBuffers &tb)
{
    size_t ny = 0, ns = 0, nc = 0;
    std::vector<DevGen> t = g;
    for (const DevGen &x : g) {
        ny += r256(envelope(x.K, x.ld_y, x.len));
        ns += r256(envelope(x.N, x.ld_s, x.len));
        nc += r256((size_t)x.K * x.N);
    }
    if (hipMalloc(reinterpret_cast<void **>(&tb.y), std::max<size_t>(ny, 256)) != hipSuccess)
        return GF_ENOMEM;
    if (p->shape_only) {
        if (hipMalloc(reinterpret_cast<void **>(&tb.s), std::max<size_t>(ns, 256)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&tb.c), std::max<size_t>(nc, 256)) != hipSuccess)
            return GF_ENOMEM;
        // coefficient 1 is a field element of every field; payload bytes are whatever is there
        if (hipMemset(tb.c, 1, std::max<size_t>(nc, 256)) != hipSuccess)
            return GF_EDEVICE;
    }
    size_t oy = 0, os = 0, oc = 0;
    for (DevGen &x : t) {
        x.Y = tb.y + oy;
        oy += r256(envelope(x.K, x.ld_y, x.len));
        if (p->shape_only) {
            x.S = tb.s + os;
            x.C = tb.c + oc;
            os += r256(envelope(x.N, x.ld_s, x.len));
            oc += r256((size_t)x.K * x.N);
        }
    }
    if (!t.empty() && hipMemcpy(p->d_bound, t.data(), t.size() * sizeof(DevGen), hipMemcpyHostToDevice) != hipSuccess)
        return GF_EDEVICE;
    return GF_OK;
}

// The autotuner: every schedule candidate (kernel form, and for the vector-ALU
// forms the payload bytes per lane) is timed on the batch's own shapes, the
// median of three launches each; the fastest then also tries 3/4 and 1/2 of
// the full persistent grid.  A candidate replaces the current best only when
// it is more than 3% faster, so near-ties resolve the same way every time.
// The choice is cached per class of batch (gf_tune.cpp).
static int autotune(gf_plan *p, DevState *d, const std::vector<DevGen> &g, const gf_tuning *tune)
{
    const std::string key = tune_key(p->field, g, p->src_aligned4, 0, tune ? tune->bytes_per_lane : 0,
                                     tune ? tune->grid_blocks : 0);
    TuneChoice c;
    if (tune_cache_get(key, &c) && (c.form != 3 || p->field <= 4) && (c.form < 4 || p->small_ok)) {
        p->tuned_from_cache = true;
        p->fixed_D = (tune && tune->bytes_per_lane) ? tune->bytes_per_lane / 4 : c.fixed_D;
        return make_schedule(p, d, g, c.form, tune, c.grid_pct);
    }
    TrialBuffers tb;
    int rc = trial_table(p, g, tb);
    if (rc)
        return rc;
    struct Cand {
        int form, D;
    };
    std::vector<Cand> cands;
    const bool fixed_bpl = tune && tune->bytes_per_lane;
    const int D0 = fixed_bpl ? tune->bytes_per_lane / 4 : 0;
    cands.push_back({p->src_aligned4 ? 2 : 1, p->src_aligned4 ? 0 : D0});   // the rule's choice first
    for (int D : fixed_bpl ? std::vector<int>{D0} : std::vector<int>{0, 4, 2, 1})
        cands.push_back({1, D});
    cands.push_back({2, 0});
    if (p->small_ok) {
        cands.push_back({4, 0});
        cands.push_back({5, 0});
    }
    if (p->field <= 4)
        for (int D : fixed_bpl ? std::vector<int>{D0} : std::vector<int>{0, 4})
            cands.push_back({3, D});
    TuneChoice best{0, 0, 100, -1};
    auto consider = [&](int form, int D, int pct) -> int {
        for (const TuneChoice &t : p->trials)
            if (t.form == form && t.fixed_D == D && t.grid_pct == pct)
                return GF_OK;   // already timed
        p->fixed_D = D;
        int r = make_schedule(p, d, g, form, tune, pct);
        if (r)
            return r;
        const double ms = time_schedule(p, d, p->d_bound);
        p->trials.push_back(TuneChoice{form, D, pct, ms});
        if (ms > 0 && (best.ms < 0 || ms < 0.97 * best.ms))
            best = TuneChoice{form, D, pct, ms};
        return GF_OK;
    };
    for (const Cand &x : cands)
        if ((rc = consider(x.form, x.D, 100)))
            return rc;
    if (best.ms < 0)
        return GF_EDEVICE;
    if (!(tune && tune->grid_blocks != 0) && best.form != 5) {
        const TuneChoice top = best;
        // the vector-ALU forms also without persistence: a wave per tile
        if ((top.form == 1 || top.form == 3) && (rc = consider(top.form, top.fixed_D, 0)))
            return rc;
        // smaller grids while they keep winning: memory-bound forms can run
        // faster with fewer waves in flight; stop two steps past the best
        if (best.grid_pct != 0) {
            for (int pct : {75, 50, 35, 25, 18}) {
                if ((rc = consider(top.form, top.fixed_D, pct)))
                    return rc;
                if (3 * pct < 2 * best.grid_pct)
                    break;
            }
        }
    }
    p->fixed_D = best.fixed_D;
    if ((rc = make_schedule(p, d, g, best.form, tune, best.grid_pct)))
        return rc;
    if (hipDeviceSynchronize() != hipSuccess)
        return GF_EDEVICE;
    tune_cache_put(key, best);
    return GF_OK;
}

// form: 1 table, 2 bit-matrix, 3 bit-plane (n <= 4), 4 and 5 the small-generation
// streaming forms (queued, chunked); 0 = time each on the
// plan's own data and keep the fastest (only when `may_run` allows launching
// before the caller asks).
static int build_encode_schedule(gf_plan *p, const std::vector<DevGen> &gens, const gf_tuning *tune, bool may_run)
{
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    if (tune && tune->bytes_per_lane) {
        if (tune->bytes_per_lane != 4 && tune->bytes_per_lane != 8 && tune->bytes_per_lane != 16)
            return GF_EINVAL;
        p->fixed_D = tune->bytes_per_lane / 4;
    }
    int form = tune ? tune->form : 0;
    if (form < 0 || form > 5 || (form == 3 && p->field > 4))
        return GF_EINVAL;
    // grid_blocks -1: a workgroup per four wave tiles, for the forms that have it
    if (tune && (tune->grid_blocks < -1 || (tune->grid_blocks == -1 && form != 1 && form != 3 && form != 5)))
        return GF_EINVAL;
    std::vector<DevGen> g = gens;
    p->src_aligned4 = true;
    bool mf_ok = true;   // the bit-matrix kernels count a tile's steps in 32 bits
    p->small_ok = true;  // every generation fits the streaming form
    for (DevGen &x : g) {
        p->small_max = std::max<int>(p->small_max, (int)std::max(x.K, x.N));
        if (x.len > (1ull << 34))
            mf_ok = false;
        x.align = row_align(x.S, x.N > 1 ? x.ld_s : 0, x.Y, x.K > 1 ? x.ld_y : 0);
        if (x.K > STREAM_MAX || x.N > STREAM_MAX || x.align < 16)   // the streaming form reads 16-byte blocks
            p->small_ok = false;
        if ((((uintptr_t)x.S) | (x.N > 1 ? x.ld_s : 0)) % 4 != 0)
            p->src_aligned4 = false;
    }
    if ((rc = upload(&p->d_gens, g)))
        return rc;
    const unsigned err_init[2] = {0, 1};
    if (!g.empty() &&
        hipMalloc(reinterpret_cast<void **>(&p->d_bound), g.size() * sizeof(DevGen)) != hipSuccess)
        return GF_ENOMEM;
    if (hipMalloc(reinterpret_cast<void **>(&p->d_err), sizeof err_init) != hipSuccess)
        return GF_ENOMEM;
    if (hipMemcpy(p->d_err, err_init, sizeof err_init, hipMemcpyHostToDevice) != hipSuccess)
        return GF_EDEVICE;
    if (hipMalloc(reinterpret_cast<void **>(&p->d_ctr), GF_QUEUE_CTR_WORDS * sizeof(unsigned)) != hipSuccess)
        return GF_ENOMEM;
    if (hipMemset(p->d_ctr, 0, GF_QUEUE_CTR_WORDS * sizeof(unsigned)) != hipSuccess)
        return GF_EDEVICE;
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
        return GF_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess)
        return GF_EDEVICE;
    if (form == 2 && !mf_ok)
        return GF_ERANGE;
    if (form >= 4 && !p->small_ok)
        return GF_EINVAL;
    if (form == 0 && (!may_run || !mf_ok))   // no trial launches: the bit-matrix form when its DMA path applies
        form = p->src_aligned4 && mf_ok ? 2 : 1;
    if (form != 0)
        return make_schedule(p, d, g, form, tune);
    return autotune(p, d, g, tune);
}

static int plan_encode_impl(int field, const gf_gen *gens, int count, const gf_tuning *tune, gf_plan **out)
{
    if (!out)
        return GF_EINVAL;
    *out = nullptr;
    if (!valid_field(field) || count < 0 || (count > 0 && !gens))
        return GF_EINVAL;
    std::vector<DevGen> g(count);
    bool shape_only = count > 0;
    for (int i = 0; i < count; i++) {
        const gf_gen &x = gens[i];
        if (x.K > GF_MAX_K)
            return GF_ERANGE;
        const bool no_ptr = !x.C && !x.S && !x.Y;
        if (i > 0 && no_ptr != shape_only)
            return GF_EINVAL;            // all descriptors carry pointers, or none does
        shape_only = no_ptr;
        int rc;
        if (no_ptr) {
            // a shape: the rows are taken to start 16-byte aligned
            rc = check_encode_args(field, kShapeC, (int)x.K, (int)x.N, kShapeS, x.ld_s, kShapeY, x.ld_y, x.len);
        } else {
            rc = check_encode_args(field, x.C, (int)x.K, (int)x.N, x.S, x.ld_s, x.Y, x.ld_y, x.len);
        }
        if (rc)
            return rc;
        g[i] = DevGen{x.C, x.S, x.Y, x.len, x.ld_s, x.ld_y, x.K, x.N, nullptr, 0, 1};
    }
    gf_plan *p = new (std::nothrow) gf_plan;
    if (!p)
        return GF_ENOMEM;
    p->kind = 0;
    p->field = field;
    p->count = count;
    p->shape_only = shape_only;
    (void)hipGetDevice(&p->dev);
    p->gens.assign(gens, gens + count);
    int rc = build_encode_schedule(p, g, tune, true);
    if (rc) {
        plan_free_device(p);
        delete p;
        return rc;
    }
    *out = p;
    return GF_OK;
}

extern "C" {

int gf_plan_encode(int field, const gf_gen *gens, int count, const gf_tuning *tune, gf_plan **out)
{
    return plan_encode_impl(field, gens, count, tune, out);
}

// One recoding as encode descriptors.  Coefficients are single field
// elements, so the word-wise product of the encode kernels equals the element
// product on them.  When each packet is one row [coefficients | payload] in
// both input and output, header and payload are one product over N + len
// bytes (returns 1, `pay` only); otherwise the header Cout = R * Cin and the
// payload Yout = R * Bin are separate products (returns 2).
static int recode_gens(const gf_recode_desc &r, gf_gen &head, gf_gen &pay)
{
    if (r.Bin == r.Cin + r.N && r.Yout == r.Cout + r.N && r.ld_b == r.ld_cin && r.ld_y == r.ld_cout) {
        pay = gf_gen{r.R, r.Cin, r.Cout, r.Kout, r.M, r.N + r.len, r.ld_cin, r.ld_cout};
        return 1;
    }
    head = gf_gen{r.R, r.Cin, r.Cout, r.Kout, r.M, (uint64_t)r.N, r.ld_cin, r.ld_cout};
    pay = gf_gen{r.R, r.Bin, r.Yout, r.Kout, r.M, r.len, r.ld_b, r.ld_y};
    return 2;
}

// Rows `a` (la bytes) and `b` (lb bytes) share the pitch ld: they are
// disjoint when b sits in the gap after a's bytes within each row, or a in
// the gap after b's.
static bool rows_interleave(const uint8_t *a, size_t la, const uint8_t *b, size_t lb, size_t ld)
{
    const intptr_t d = (intptr_t)b - (intptr_t)a;
    return (d >= (intptr_t)la && (size_t)d + lb <= ld) || (-d >= (intptr_t)lb && (size_t)(-d) + la <= ld);
}

static int check_recode_args(int field, const gf_recode_desc &r)
{
    if (r.reserved || r.N < 1 || r.M < 1)
        return GF_EINVAL;
    if (r.N > GF_MAX_N || r.M > GF_MAX_N || r.Kout > GF_MAX_K)
        return GF_ERANGE;
    if ((r.M > 1 && r.ld_cin < r.N) || (r.Kout > 1 && r.ld_cout < r.N))
        return GF_EINVAL;
    gf_gen h, y;
    if (recode_gens(r, h, y) == 1)
        return check_encode_args(field, y.C, (int)y.K, (int)y.N, y.S, y.ld_s, y.Y, y.ld_y, y.len);
    int rc = check_encode_args(field, h.C, (int)h.K, (int)h.N, h.S, h.ld_s, h.Y, h.ld_y, h.len);
    if (!rc)
        rc = check_encode_args(field, y.C, (int)y.K, (int)y.N, y.S, y.ld_s, y.Y, y.ld_y, y.len);
    if (rc || r.Kout == 0)
        return rc;
    // each output against the other product's operands, and the two outputs
    const size_t eh = envelope(r.Kout, r.ld_cout, r.N);
    if (overlap(h.Y, eh, r.Bin, envelope(r.M, r.ld_b, r.len)))
        return GF_EINVAL;
    if (r.len) {
        const size_t ey = envelope(r.Kout, r.ld_y, r.len);
        if (overlap(y.Y, ey, r.Cin, envelope(r.M, r.ld_cin, r.N)))
            return GF_EINVAL;
        const bool apart = r.Kout == 1 ? !overlap(h.Y, r.N, y.Y, r.len)
                           : r.ld_cout == r.ld_y && rows_interleave(h.Y, r.N, y.Y, r.len, r.ld_y);
        if (!apart && overlap(y.Y, ey, h.Y, eh))
            return GF_EINVAL;
    }
    return GF_OK;
}

int gf_recode(int field, const uint8_t *R, int Kout, int M, int N, const uint8_t *Cin, size_t ld_cin,
              const uint8_t *Bin, size_t ld_b, uint8_t *Cout, size_t ld_cout, uint8_t *Yout, size_t ld_y,
              size_t len, void *stream)
{
    if (Kout < 0 || M < 1 || N < 1)
        return GF_EINVAL;
    const gf_recode_desc r{R, Cin, Bin, Cout, Yout, (uint32_t)Kout, (uint32_t)M, (uint32_t)N, 0,
                           len, ld_cin, ld_b, ld_cout, ld_y};
    int rc = check_recode_args(field, r);
    if (rc || Kout == 0)
        return rc;
    gf_gen h, y;
    if (recode_gens(r, h, y) == 2 &&
        (rc = encode_impl(field, h.C, (int)h.K, (int)h.N, h.S, h.ld_s, h.Y, h.ld_y, h.len, nullptr, nullptr, 0,
                          stream)))
        return rc;
    if (y.len == 0)
        return GF_OK;
    return encode_impl(field, y.C, (int)y.K, (int)y.N, y.S, y.ld_s, y.Y, y.ld_y, y.len, nullptr, nullptr, 0,
                       stream);
}

int gf_plan_recode(int field, const gf_recode_desc *descs, int count, const gf_tuning *tune, gf_plan **out)
{
    if (!out)
        return GF_EINVAL;
    *out = nullptr;
    if (!valid_field(field) || count < 0 || (count > 0 && !descs))
        return GF_EINVAL;
    std::vector<gf_gen> heads, pays(count);
    for (int i = 0; i < count; i++) {
        int rc = check_recode_args(field, descs[i]);
        if (rc)
            return rc;
        gf_gen h;
        if (recode_gens(descs[i], h, pays[i]) == 2)
            heads.push_back(h);
    }
    gf_plan *head = nullptr, *p = nullptr;
    int rc = heads.empty() ? GF_OK : plan_encode_impl(field, heads.data(), (int)heads.size(), tune, &head);
    if (rc)
        return rc;
    if ((rc = plan_encode_impl(field, pays.data(), count, tune, &p))) {
        gf_plan_destroy(head);
        return rc;
    }
    p->kind = 2;
    p->head = head;
    *out = p;
    return GF_OK;
}

int gf_plan_decode(int field, const gf_sys *sys, int count, const gf_tuning *tune, gf_plan **out)
{
    if (!out)
        return GF_EINVAL;
    *out = nullptr;
    if (!valid_field(field) || count < 0 || (count > 0 && !sys))
        return GF_EINVAL;
    for (int i = 0; i < count; i++) {
        const gf_sys &s = sys[i];
        if (s.N < 1 || s.reserved != 0)
            return GF_EINVAL;
        if (s.N > GF_MAX_N)
            return GF_ERANGE;
        if (!s.C || (s.len > 0 && (!s.B || !s.S || (s.N > 1 && (s.ld_b < s.len || s.ld_s < s.len)))))
            return GF_EINVAL;
        size_t es, eb, ec;
        if (!span_of(s.S, s.N, s.ld_s, s.len, &es) || !span_of(s.B, s.N, s.ld_b, s.len, &eb) ||
            !span_of(s.C, s.N, s.N, s.N, &ec))
            return GF_EINVAL;
        if (overlap(s.S, es, s.B, eb) || overlap(s.S, es, s.C, ec))
            return GF_EINVAL;
    }
    gf_plan *p = new (std::nothrow) gf_plan;
    if (!p)
        return GF_ENOMEM;
    p->kind = 1;
    p->field = field;
    p->count = count;
    (void)hipGetDevice(&p->dev);
    int rc = GF_OK;
    // inverse matrices and ranks live in the plan
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; i++)
        off[i + 1] = off[i] + (((size_t)sys[i].N * sys[i].N + 15) / 16) * 16;
    if (count > 0) {
        if (hipMalloc(reinterpret_cast<void **>(&p->d_cinv), std::max<size_t>(off[count], 16)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&p->d_rank), sizeof(int) * count) != hipSuccess)
            rc = GF_ENOMEM;
    }
    // systems grouped by size class (N <= 32, 64, 128, 256) for the elimination launches
    auto cls = [](uint32_t N) { return N <= 32 ? 0 : N <= 64 ? 1 : N <= 128 ? 2 : 3; };
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls(sys[a].N) < cls(sys[b].N); });
    std::vector<DevSys> ds(count);
    for (int j = 0; j < count; j++) {
        const int i = order[j];
        ds[j] = DevSys{sys[i].C, p->d_cinv + off[i], p->d_rank + i, sys[i].N, 0};
        p->class_count[cls(sys[i].N)]++;
    }
    for (int c = 1; c < 4; c++)
        p->class_begin[c] = p->class_begin[c - 1] + p->class_count[c - 1];
    p->sys_order = order;
    if (!rc)
        rc = upload(&p->d_sys, ds);
    for (int i = 0; i < 3 && !rc; i++)
        if (hipStreamCreateWithFlags(&p->aux[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_done[i], hipEventDisableTiming) != hipSuccess)
            rc = GF_EDEVICE;
    if (!rc && hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess)
        rc = GF_EDEVICE;
    std::vector<DevGen> g(count);
    for (int i = 0; i < count; i++) {
        const gf_sys &s = sys[i];
        g[i] = DevGen{p->d_cinv + off[i], s.B, s.S, s.len, s.ld_b, s.ld_s, s.N, s.N, p->d_rank + i, (int)s.N, 1};
    }
    // one product schedule per size class, so that a class's product can follow
    // its own elimination while larger classes are still being eliminated; the
    // plan reports the schedule of its largest class
    for (int c = 0; c < 4 && !rc; c++) {
        if (p->class_count[c] == 0)
            continue;
        std::vector<DevGen> gc;
        for (int j = p->class_begin[c]; j < p->class_begin[c] + p->class_count[c]; j++)
            gc.push_back(g[order[j]]);
        gf_plan *q = new (std::nothrow) gf_plan;
        if (!q) {
            rc = GF_ENOMEM;
            break;
        }
        q->field = field;
        q->dev = p->dev;
        q->count = (int)gc.size();
        p->prod[c] = q;
        if (!(rc = build_encode_schedule(q, gc, tune, false))) {
            p->form = q->form;
            p->grid = q->grid;
            p->fixed_D = q->fixed_D;
        }
    }
    if (!rc && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
        rc = GF_EDEVICE;
    if (rc) {
        plan_free_device(p);
        delete p;
        return rc;
    }
    *out = p;
    return GF_OK;
}

// A plan's device buffers belong to the device that was current when it was
// made; it runs only while that device is current.
static int plan_device_ok(const gf_plan *p)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return GF_EDEVICE;
    return dev == p->dev ? GF_OK : GF_EINVAL;
}

static int run_plan(gf_plan *p, int *d_rank, hipStream_t s)
{
    DevState *d;
    int rc = plan_device_ok(p);
    if (rc || (rc = current_state(&d)))
        return rc;
    const int f = p->field;
    if (p->head && (rc = run_plan(p->head, nullptr, s)))
        return rc;
    if (p->kind == 1) {
        // the size classes run side by side, each its elimination and then its
        // product: the largest on `s`, the others on the plan's own streams,
        // forked from and joined back to `s`
        static const int kClassN[4] = {32, 64, 128, 256};
        int classes = 0;
        for (int c = 0; c < 4; c++)
            classes += p->class_count[c] > 0;
        if (classes > 1 && hipEventRecord(p->ev_fork, s) != hipSuccess)
            return GF_EDEVICE;
        int used = 0;
        for (int c = 3; c >= 0; c--) {
            if (p->class_count[c] == 0)
                continue;
            hipStream_t on = used == 0 ? s : p->aux[used - 1];
            if (used > 0 && hipStreamWaitEvent(on, p->ev_fork, 0) != hipSuccess)
                return GF_EDEVICE;
            hipError_t e = launch_invert(p->d_sys + p->class_begin[c], p->class_count[c], nullptr, kClassN[c], nullptr,
                                         nullptr, field_ptab(d, f), field_inv(d, f), on);
            if (e != hipSuccess)
                return GF_EDEVICE;
            if ((rc = launch_schedule(p->prod[c], d, on)))
                return rc;
            if (used > 0 && (hipEventRecord(p->ev_done[used - 1], on) != hipSuccess ||
                             hipStreamWaitEvent(s, p->ev_done[used - 1], 0) != hipSuccess))
                return GF_EDEVICE;
            used++;
        }
    } else if ((rc = launch_schedule(p, d, s))) {
        return rc;
    }
    if (p->kind == 1 && d_rank && p->count > 0)
        if (hipMemcpyAsync(d_rank, p->d_rank, sizeof(int) * p->count, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return GF_EDEVICE;
    return GF_OK;
}

int gf_plan_launch(gf_plan *p, int *d_rank, void *stream)
{
    if (!p || p->shape_only)
        return GF_EINVAL;
    return run_plan(p, p->kind == 1 ? d_rank : nullptr, (hipStream_t)stream);
}

int gf_encode_batched(int field, const gf_gen *d_gens, int count, gf_plan *p, void *stream)
{
    if (!p || p->kind == 1 || field != p->field || count != p->count)
        return GF_EINVAL;
    if (!d_gens)
        return gf_plan_launch(p, nullptr, stream);
    if (p->kind != 0)
        return GF_EINVAL;    // recode plans run on their own descriptors
    DevState *d;
    int rc = plan_device_ok(p);
    if (rc || (rc = current_state(&d)))
        return rc;
    if (count == 0)
        return GF_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (launch_bind_gens(d_gens, p->d_gens, p->d_bound, count, p->d_err,
                         reinterpret_cast<const int *>(p->d_err + 1), s) != hipSuccess)
        return GF_EDEVICE;
    return launch_schedule(p, d, s, p->d_bound);
}

int gf_plan_errors(gf_plan *p, uint64_t *out)
{
    if (!p || !out)
        return GF_EINVAL;
    if (int rc = plan_device_ok(p))
        return rc;
    unsigned v = 0;
    const unsigned zero = 0;
    if (!p->d_err) {   // a decode plan: no descriptors are bound to it
        *out = 0;
        return GF_OK;
    }
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&v, p->d_err, sizeof v, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(p->d_err, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
        return GF_EDEVICE;
    *out = v;
    return GF_OK;
}

int gf_decode_batched(int field, const gf_sys *d_sys, int count, int *d_rank, void *ws, size_t ws_bytes,
                      void *stream)
{
    if (!valid_field(field) || count < 0)
        return GF_EINVAL;
    if (count == 0)
        return GF_OK;
    if (!d_sys || !ws || (uintptr_t)ws % 256 != 0)
        return GF_EINVAL;
    const DecWsLayout L = dec_ws_layout((size_t)count);
    if (ws_bytes < L.fixed || (ws_bytes - L.fixed) / (size_t)count < 256)
        return GF_EINVAL;
    const uint64_t slot = ((ws_bytes - L.fixed) / (size_t)count) / 256 * 256;
    size_t ew, es;
    if (!span_of(ws, 1, 0, ws_bytes, &ew) || !span_of(d_sys, 1, 0, (size_t)count * sizeof(gf_sys), &es) ||
        overlap(ws, ew, d_sys, es) || (d_rank && overlap(ws, ew, d_rank, (size_t)count * sizeof(int))))
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    DecSched w;
    w.cls_count = reinterpret_cast<unsigned *>(w8 + L.hdr);
    w.bounds = w.cls_count + 4;
    w.ctr = reinterpret_cast<unsigned *>(w8 + L.ctr);
    w.lists = reinterpret_cast<DevSys *>(w8 + L.lists);
    w.gens = reinterpret_cast<DevGen *>(w8 + L.gens);
    w.tiles = reinterpret_cast<DevTile *>(w8 + L.tiles);
    w.tile_cap = L.tile_cap;
    w.rank = d_rank ? d_rank : reinterpret_cast<int *>(w8 + L.rank);
    w.inv = w8 + L.fixed;
    w.slot = slot;
    const hipStream_t s = (hipStream_t)stream;
    if (launch_dec_schedule(d_sys, count, w, s) != hipSuccess)
        return GF_EDEVICE;
    static const int kClassN[4] = {32, 64, 128, 256};
    for (int c = 3; c >= 0; c--)
        if (launch_invert(w.lists + (size_t)c * count, count, nullptr, kClassN[c], nullptr, nullptr,
                          field_ptab(d, field), field_inv(d, field), s, w.cls_count + c) != hipSuccess)
            return GF_EDEVICE;
    // the product: systems with 4-byte aligned coded rows on the direct-to-LDS
    // kernel, the others on the byte-load one (a kernel with an empty queue
    // has every workgroup leave at once)
    const int grid_dma = d->cus * encode_mfma_blocks_per_cu(true);
    if (launch_encode_mfma(w.gens, w.tiles, nullptr, w.bounds, 1, w.ctr, grid_dma, field_rows(d, field), true, s) !=
            hipSuccess ||
        launch_encode_mfma(w.gens, w.tiles + L.tile_cap, nullptr, w.bounds + MF_QUEUES + 1, 1,
                           w.ctr + GF_QUEUE_CTR_WORDS, d->cus, field_rows(d, field), false, s) != hipSuccess)
        return GF_EDEVICE;
    return GF_OK;
}

int gf_plan_launch_graph(gf_plan *p, int *d_rank, void *stream)
{
    if (!p || p->shape_only)
        return GF_EINVAL;
    if (int rc = plan_device_ok(p))
        return rc;
    if (p->exec && p->graph_rank != d_rank) {
        (void)hipGraphExecDestroy(p->exec);
        (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
    if (!p->exec) {
        if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return GF_EDEVICE;
        int rc = run_plan(p, p->kind == 1 ? d_rank : nullptr, p->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap, &g);
        if (rc) {
            if (g)
                (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g)
            return GF_EDEVICE;
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return GF_EDEVICE;
        }
        p->graph = g;
        p->exec = x;
        p->graph_rank = d_rank;
    }
    return dev_err(hipGraphLaunch(p->exec, (hipStream_t)stream));
}

int gf_ceiling(int what, void *d_buf, size_t bytes, int blocks, int iters, void *stream)
{
    if (what < 0 || what > 4 || !d_buf || blocks < 1 || iters < 0)
        return GF_EINVAL;
    if (what == 0 || what == 4 ? bytes < 64 : bytes < (size_t)blocks * 256 * sizeof(uint32_t))
        return GF_EINVAL;
    DevState *d;
    int rc = current_state(&d);
    if (rc)
        return rc;
    return dev_err(launch_ceiling(what, d_buf, bytes, blocks, iters, (hipStream_t)stream));
}

int gf_plan_tuning(const gf_plan *p, gf_tuning *out)
{
    if (!p || !out)
        return GF_EINVAL;
    out->form = p->form;
    out->bytes_per_lane = 4 * p->fixed_D;
    out->grid_blocks = p->grid;
    out->reserved = 0;
    return GF_OK;
}

void gf_plan_destroy(gf_plan *p)
{
    if (!p)
        return;
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != p->dev && hipSetDevice(p->dev) == hipSuccess;
    (void)hipDeviceSynchronize();
    plan_free_device(p);
    if (other)
        (void)hipSetDevice(cur);
    delete p;
}

}  // extern "C"
