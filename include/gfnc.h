/*
 * gfnc.h -- GF(2^n) random linear network coding on AMD Instinct MI355X (gfx950).
 *
 * A C ABI over hand-written HIP kernels.  The operations follow
 * Guenther, Appel, Carle, "Galois Field Arithmetics for Linear Network Coding
 * using AVX 512 Instruction Set Extensions" (arXiv 1909.02871):
 *
 *   - a packet of l bits is a sequence of M = l/n words of n bits, each an
 *     element of GF(q), q = 2^n, n in {1, 2, 4, 8}                 (Sec. II)
 *   - encoding: a coded packet is the sum over the generation's N source
 *     packets of c_i times packet i, i.e. a matrix-vector product  (Sec. II, Eq. 1)
 *   - madd: multiply a region by a constant and add (XOR) it into an
 *     accumulator region; c = 0 is a no-op, c = 1 a plain XOR      (Sec. II, Sec. IV)
 *   - decoding (Sec. I mentions that a generation can fail to decode) is
 *     Gauss-Jordan elimination of the coefficient matrix.
 *
 * Field polynomials (the paper names none): GF(4) x^2+x+1, GF(16) x^4+x+1,
 * GF(256) x^8+x^4+x^3+x^2+1; GF(2) multiplication is AND.
 *
 * Conventions for every call
 *   - Pointers named d_* or documented as "device" are device memory (e.g.
 *     hipMalloc'd or a torch CUDA tensor's data pointer); the caller owns
 *     them.  Host arrays are documented as such.
 *   - Payload is uint8 bytes holding 8/n words each; word k of a byte is
 *     bits [n*k, n*k+n).  Coefficients are one field element per byte (< q).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every compute
 *     call only enqueues work on `stream` and returns; results are visible
 *     after the stream is synchronised.
 *   - Return value: GF_OK (0) or a negative GF_E* code.  Argument errors are
 *     detected before anything is enqueued; nothing is written then.
 *   - Lengths are in bytes; any length >= 0 and any alignment is accepted
 *     (16-byte-aligned rows take the fast path).  len = 0 is a no-op.
 */
#ifndef GFNC_H
#define GFNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Field selector: the value is the number of bits per word, n. */
typedef enum { GF_2 = 1, GF_4 = 2, GF_16 = 4, GF_256 = 8 } gf_field;

enum {
    GF_OK = 0,
    GF_EINVAL = -1,      /* bad argument: field, coefficient >= q, size, null, overlap, or a
                            buffer span ((rows - 1) * pitch + len) past the address space */
    GF_ENOTINIT = -2,    /* library could not initialise its tables */
    GF_EDEVICE = -3,     /* a HIP runtime call failed */
    GF_ESINGULAR = -4,   /* coefficient matrix not invertible: not returned by the asynchronous
                            calls (they write the rank to d_rank); for callers that synchronise
                            and find rank < N */
    GF_ENOMEM = -5,      /* device or host allocation failed (plan and server creation, serving steps) */
    GF_ERANGE = -6,      /* size above a documented limit */
    GF_ECANCELED = -7    /* serving: the request was cancelled before it completed */
};

/* Initialise the field tables on the current device.  Idempotent and
 * thread-safe; called implicitly by every entry point.  Returns GF_OK or
 * GF_EDEVICE. */
int gf_init(void);

/* Static text for a GF_* code. */
const char *gf_strerror(int code);

/* Largest generation size N accepted by encode and decode. */
#define GF_MAX_N 256
/* Most coded rows of one generation in a batched plan or a serving request
 * (GF_ERANGE above it; a single gf_encode has no such limit). */
#define GF_MAX_K 65535

/* ----------------------------------------------------------- region ops
 * madd (Sec. II; the shuffle kernel of Sec. IV-A, Algorithm 1):
 *     y[j] := y[j] + c * x[j]   for every word of the len bytes.
 * c = 0 enqueues nothing; c = 1 is a plain XOR.  y == x (exact alias) is
 * allowed and gives (1 + c) * x; any other overlap is GF_EINVAL.
 * y, x: device, len bytes each.  c < q (GF(2): c in {0, 1}). */
int gf_region_madd(int field, uint8_t *y, const uint8_t *x, int c, size_t len, void *stream);

/* y[j] := c * x[j] (y == x allowed, other overlap GF_EINVAL).  c = 0 zero-fills y. */
int gf_region_mul(int field, uint8_t *y, const uint8_t *x, int c, size_t len, void *stream);

/* One region of a batched madd.  y, x are device pointers. */
typedef struct {
    uint8_t *y;
    const uint8_t *x;
    uint64_t len;
    uint32_t c;
    uint32_t reserved;   /* must be 0 */
} gf_region;

/* Many independent madds (Sec. II) in one launch.
 * d_regions: device array of `count` gf_region; every len <= max_len.
 * Regions must not overlap one another (a region may alias its own x).
 * The descriptors are not validated on the host (they live on the device);
 * a coefficient >= q is treated as 0 by the kernel. */
int gf_region_madd_batched(int field, const gf_region *d_regions, int count, size_t max_len,
                           void *stream);

/* --------------------------------------------------------------- encode
 * Eq. (1) for K coding vectors at once:
 *     Y[k][j] = sum_{i<N} C[k][i] * S[i][j],   k < K, j < len,
 * a product of the K x N coefficient matrix with the generation.
 * C: device, K x N row-major, one element per byte.  Entries must be < q:
 *    device matrices are not checked, and what an entry >= q contributes
 *    depends on the kernel form.
 * S: device, N rows of len bytes, row i at S + i*ld_s (ld_s >= len).
 * Y: device, K rows, row k at Y + k*ld_y (ld_y >= len); overwritten.
 * Y must not overlap S or C.  1 <= N <= GF_MAX_N, K >= 0. */
int gf_encode(int field, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s,
              uint8_t *Y, size_t ld_y, size_t len, void *stream);

/* --------------------------------------------------------------- decode
 * Gauss-Jordan decoding of one generation: S = C^-1 B.
 * The argument order follows the madd signature of Sec. IV-A (operands, then
 * the destination with its pitch, then the byte length).
 * C: device, N x N coefficient rows of the N received coded packets.
 * B: device, N coded packets, row i at B + i*ld_b.
 * S: device output, row i at S + i*ld_s; written only if C is invertible.
 * ws: device workspace of at least gf_decode_workspace(field, N, 1) bytes
 *     (it receives C^-1, and the rank when d_rank is NULL).
 * d_rank: device int (may be NULL); receives rank(C).  The call returns
 * GF_OK once enqueued; rank < N means singular and S untouched.
 * 1 <= N <= GF_MAX_N (GF_ERANGE above). */
int gf_decode(int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, uint8_t *S, size_t ld_s,
              size_t len, void *ws, size_t ws_bytes, int *d_rank, void *stream);

/* Device workspace in bytes for decoding `count` systems of at most max_N
 * source packets each: count * (max_N^2 rounded up to 256) plus 256-byte
 * rounded room for count ranks.  0 for a bad field, max_N outside
 * [1, GF_MAX_N] or count < 1. */
size_t gf_decode_workspace(int field, int max_N, int count);

/* gf_decode without the workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  It allocates nothing: C^-1, and the rank when
 * d_rank is NULL, go to a fixed scratch array in the library's device memory
 * of GF_MAX_N^2 + 256 bytes (64.25 KiB), one per device, held until the
 * process ends.  gf_init() must have run with this device current (else
 * GF_ENOTINIT).  Every call on a device shares its scratch array, so calls
 * that overlap on one device (other streams, other threads) race: serialise
 * them, e.g. on one stream.  Arguments, errors and results as gf_decode;
 * N > GF_MAX_N is GF_ERANGE. */
int gf_decode_noalloc(int field, const uint8_t *C, const uint8_t *B, size_t ld_b, int N, uint8_t *S,
                      size_t ld_s, size_t len, int *d_rank, void *stream);

/* Invert one N x N matrix: Cinv (device, N x N) := C^-1; *d_rank := rank(C).
 * Cinv is written only if C is invertible.  Uses no workspace. */
int gf_invert(int field, const uint8_t *C, int N, uint8_t *Cinv, int *d_rank, void *stream);

/* ----------------------------------------------------- batched calls
 * Many uneven generations in one launch.  The batched calls read their
 * descriptors from DEVICE memory when they run, so the same call serves new
 * buffers without host work, allocates nothing and can be captured in a HIP
 * graph.  The descriptors are not validated on the host (they live on the
 * device): every generation must obey the rules of gf_encode / gf_decode
 * (pitches >= len, outputs disjoint from every input and from each other,
 * entries < q), and what the kernels can check they do (see each call). */
typedef struct {
    const uint8_t *C;   /* device, K x N */
    const uint8_t *S;   /* device, N rows, ld_s apart */
    uint8_t *Y;         /* device, K rows, ld_y apart */
    uint32_t K, N;
    uint64_t len, ld_s, ld_y;
} gf_gen;

typedef struct {
    const uint8_t *C;   /* device, N x N */
    const uint8_t *B;   /* device, N coded rows, ld_b apart */
    uint8_t *S;         /* device, N decoded rows, ld_s apart */
    uint32_t N, reserved;
    uint64_t len, ld_b, ld_s;
} gf_sys;

/* Kernel schedule knobs.  Zero fields mean "chosen by the library".
 * form 1: byte-select table lookups on the vector ALUs.
 * form 2: the product as a GF(2) bit-matrix multiply on the matrix cores;
 *         packets longer than 2^34 bytes are rejected with GF_ERANGE.
 * form 3: bit planes on the vector ALUs, GF(2), GF(4) and GF(16) only (the
 *         coefficient split into its bits, Sec. IV-B's decomposition; one
 *         3-input bit operation per row, source, plane and dword);
 *         GF_EINVAL for GF(256).
 * form 4: small generations streamed at 16 payload bytes per lane, every
 *         generation's K x N tables staged once per tile and the strips read
 *         in bursts of about 8 KiB per wave; only when every generation has
 *         K <= 8 and N <= 8 and its rows (S, Y, ld_s, ld_y) are 16-byte
 *         aligned (GF_EINVAL otherwise).
 * form 5: form 4's generations without work queues: one wave per run of
 *         at most about 8 KiB of one generation's strips, one workgroup per
 *         four runs, as many workgroups as runs need (grid_blocks ignored);
 *         the same conditions as form 4.
 * form 0 on an encode plan: every form that applies is timed while the plan
 * is created, on the plan's own sources (a plan of shapes: on scratch inputs
 * of its shapes) into scratch outputs, so the caller's outputs are not
 * written; the fastest is kept (form 2 is skipped if a packet is too long for
 * it), then tried without persistence (forms 1 and 3) and on smaller
 * persistent grids.  The choice is cached per class of batch.  On a decode
 * plan form 0 means form 2 when every coded row starts 4-byte aligned, else 1. */
typedef struct {
    int form;           /* 0 auto, 1 table, 2 bit-matrix, 3 bit-plane, 4 small-generation stream,
                           5 small-generation chunks */
    int bytes_per_lane; /* 0 = per tile; else 4, 8 or 16 payload bytes per lane everywhere */
    int grid_blocks;    /* persistent workgroups; 0 = as many as fit on the GPU at once (or, with form
                           0, what the autotuner picks); -1 = forms 1 and 3 not persistent: a
                           workgroup per four wave tiles (GF_EINVAL for forms 2 and 4) */
    int reserved;       /* must be 0 */
} gf_tuning;

/* A plan is the tuned schedule (tiles, work queues, kernel form) of a list of
 * generation shapes.  Creating one allocates and synchronises; launching one
 * does neither.  A plan runs on the device that was current when it was
 * created (GF_EINVAL with another device current).  Launches of one plan
 * share its work-queue counters and tables, so they must not overlap: launch
 * a plan again only on the same stream, or after the previous launch has
 * completed. */
typedef struct gf_plan gf_plan;

/* gens: HOST array of `count` descriptors giving the shapes (K, N, len,
 * ld_s, ld_y).  Their pointers are either all present (device memory: the
 * plan can then run on them with gf_plan_launch, and form 0 is tuned on them)
 * or all NULL (a plan for shapes only: rows are taken to start 16-byte
 * aligned, and it runs only through gf_encode_batched). */
int gf_plan_encode(int field, const gf_gen *gens, int count, const gf_tuning *tune,
                   gf_plan **out);

/* Eq. (1) for every generation of d_gens in one persistent launch of the
 * plan's schedule (Sec. II; the madd of Sec. IV-A, Alg. 1, per coefficient).
 * d_gens: DEVICE array of `count` descriptors, count == the plan's count,
 * field == the plan's field.  d_gens[i] must have the shape of the plan's
 * i-th generation and rows at least as aligned as the plan assumed; a
 * descriptor that differs (or lacks a pointer) is skipped, its output left
 * as it was, and counted for gf_plan_errors.  d_gens NULL runs the plan on
 * the pointers it was made with (as gf_plan_launch).  Allocates nothing. */
int gf_encode_batched(int field, const gf_gen *d_gens, int count, gf_plan *plan, void *stream);

/* Descriptors gf_encode_batched skipped since the last call (synchronises the
 * device; the count is then reset). */
int gf_plan_errors(gf_plan *plan, uint64_t *out);

/* Gauss-Jordan decoding of `count` systems, S_i = C_i^-1 B_i, read from the
 * DEVICE array d_sys when the work runs, with no plan: the device sorts the
 * systems into size classes for the elimination and lays out the product's
 * work queues itself, all inside `ws`.
 * ws: device workspace, 256-byte aligned, of at least
 *     gf_decode_workspace(field, max_N, count) bytes, where max_N bounds every
 *     N; it is overwritten.
 * d_rank: device, `count` ints (may be NULL): rank(C_i); a singular system's
 *     S_i is left untouched, and a system the kernels reject (N outside
 *     [1, max_N the workspace allows], a pitch < len, a NULL pointer, or
 *     len > 2^34) gets rank -1 and no output.
 * Allocates nothing; every launch goes on `stream`. */
int gf_decode_batched(int field, const gf_sys *d_sys, int count, int *d_rank, void *ws, size_t ws_bytes,
                      void *stream);

/* A decode plan: the same decoding for a fixed list of systems (sys: HOST
 * array with device pointers), with the size classes' eliminations running
 * side by side on the plan's own streams; it owns its inverses and ranks. */
int gf_plan_decode(int field, const gf_sys *sys, int count, const gf_tuning *tune,
                   gf_plan **out);

/* Run a plan on the descriptors it was made with (encode, recode or decode;
 * d_rank: device, `count` ints, for a decode plan, may be NULL; ignored
 * otherwise).  GF_EINVAL for a plan made from shapes alone. */
int gf_plan_launch(gf_plan *plan, int *d_rank, void *stream);
/* Same work as gf_plan_launch, replayed from a HIP graph captured on first
 * use (d_rank must be the same pointer on every replay of a decode plan). */
int gf_plan_launch_graph(gf_plan *plan, int *d_rank, void *stream);
/* The schedule the plan uses (after autotuning); grid_blocks is the number of
 * workgroups a launch starts (for the non-persistent dispatches, one per four
 * wave tiles or runs). */
int gf_plan_tuning(const gf_plan *plan, gf_tuning *out);
void gf_plan_destroy(gf_plan *plan);

/* Diagnostic microbenchmarks for roofline reports (no part of the coding
 * path): what 0 copies the first half of d_buf (bytes long) to the second half
 * with 16-byte non-temporal accesses (blocks x 256 threads, grid-stride); what
 * 1 runs the table form's inner step (byte-select lookups and 3-input XORs on
 * register data: 8 coded rows x 2 sources x 4 bytes = 64 byte-madds per thread
 * and iteration), 2 back-to-back FP4 32x32x64 MFMAs (8 per wave and
 * iteration), 3 the bit-plane form's step (64 three-input bit operations per
 * thread and iteration), each on blocks x 256 threads for `iters` iterations,
 * writing one word per thread to d_buf (bytes >= blocks * 1024); what 4
 * makes what 0's copy with one workgroup per 16 KiB instead of a grid-stride
 * loop (blocks must be >= 1 and is otherwise unused, as is iters).  Time it on
 * `stream` with events. */
int gf_ceiling(int what, void *d_buf, size_t bytes, int blocks, int iters, void *stream);

/* Per-generation launches of the same work (the unbatched baseline): one
 * gf_encode per descriptor, on `stream`.  gens is a HOST array. */
int gf_encode_each(int field, const gf_gen *gens, int count, const gf_tuning *tune, void *stream);

/* ------------------------------------------------------------ recoding
 * A node in the network sends linear combinations of coded packets it has
 * received (Sec. I), without decoding them first.  Its M received packets
 * carry coefficient vectors Cin (M x N, over the generation's N source
 * packets) and payloads Bin; with a local Kout x M matrix R it sends
 *     Cout = R * Cin   (Kout x N: the new packets' coefficient vectors)
 *     Yout = R * Bin   (Kout payloads of len bytes)
 * so that Yout = Cout * S still holds for the generation's sources S, and a
 * receiver decodes recoded packets exactly like encoded ones.
 * R: device, Kout x M row-major.  Cin: M rows of N elements, ld_cin apart;
 * Cout: Kout rows of N, ld_cout apart; Bin: M rows of len bytes, ld_b apart;
 * Yout: Kout rows, ld_y apart (outputs overwritten).  Entries of R and Cin are
 * field elements (< q).  Outputs must not overlap inputs or each other.
 * 1 <= M <= GF_MAX_N, 1 <= N <= GF_MAX_N, Kout >= 0.
 * Packet layout: when every packet is one row holding its coefficient vector
 * followed by its payload (Bin == Cin + N, Yout == Cout + N, ld_b == ld_cin,
 * ld_y == ld_cout), header and payload are one product over N + len bytes;
 * otherwise the header product is enqueued first, then the payload's. */
int gf_recode(int field, const uint8_t *R, int Kout, int M, int N, const uint8_t *Cin, size_t ld_cin,
              const uint8_t *Bin, size_t ld_b, uint8_t *Cout, size_t ld_cout, uint8_t *Yout, size_t ld_y,
              size_t len, void *stream);

typedef struct {
    const uint8_t *R;     /* device, Kout x M */
    const uint8_t *Cin;   /* device, M coefficient rows, ld_cin apart */
    const uint8_t *Bin;   /* device, M payload rows, ld_b apart */
    uint8_t *Cout;        /* device, Kout coefficient rows, ld_cout apart */
    uint8_t *Yout;        /* device, Kout payload rows, ld_y apart */
    uint32_t Kout, M, N, reserved;   /* reserved must be 0 */
    uint64_t len, ld_cin, ld_b, ld_cout, ld_y;
} gf_recode_desc;

/* Plan for many recodings at once (descs: HOST array).  Launched with
 * gf_plan_launch or gf_plan_launch_graph: one persistent launch over the
 * headers that are not stored in front of their payloads (if any), then one
 * over the payloads (with the headers that are), each autotuned like
 * gf_plan_encode (form 0 times its trials on scratch outputs).
 * gf_plan_tuning reports the payload launch's schedule. */
int gf_plan_recode(int field, const gf_recode_desc *descs, int count, const gf_tuning *tune, gf_plan **out);

/* ------------------------------------------------------------ serving
 * Continuous batching of encode and decode requests on one device.
 *
 * Encode request: K coded packets Y = C * S of a generation (Eq. 1).
 * Decode request: a generation of N packets of len bytes that is rebuilt
 * from coded packets pushed one by one (coefficient vector + payload, in any
 * order, with losses).  The server keeps, in device memory, the reduced row
 * echelon form of the innovative coefficient vectors received so far; a
 * packet whose vector reduces to zero is dropped (counted); at rank N the
 * source packets are S = Csel^-1 * Bsel over the innovative packets.
 *
 * Memory: the server owns one device arena of budget_bytes.  A request is
 * admitted (FIFO; the queue waits at its head) once a service slot and its
 * working set are free: encode K * ld bytes for its output; decode about
 * 3 N^2 + 2 N * ld bytes of state and output, ld = len rounded up to 16.
 * Inputs (C, S, packets) stay in caller-owned device memory and must be
 * ready (their producing stream synchronised) before they are submitted or
 * pushed, and stay valid until the request completes.
 *
 * Time: `now` and `release` are caller clock readings in seconds; a packet is
 * used once a step runs at or after its release time.  Completion time is
 * the `now` of the call that observed it.
 *
 * Calls on one server may come from several threads; an internal mutex
 * serialises them.  A completed request's output (device, `out` with row
 * pitch `ld_out`) stays valid until gf_serve_release.
 *
 * Errors: argument errors are returned and change nothing.  A device or
 * memory failure inside gf_serve_step or gf_serve_drain (GF_EDEVICE,
 * GF_ENOMEM) can leave requests taken off their queues but never launched,
 * so the server keeps that code: every later submit, push, step and drain
 * returns it, while poll, copy_out, release and stats still serve what had
 * completed; destroy the server to recover. */
typedef struct gf_server gf_server;

typedef struct {
    int field;              /* GF_2 .. GF_256 */
    int max_slots;          /* requests in service at once; 0 = 1024 */
    int burst;              /* packets one decode request absorbs per step; 0 = 64 */
    int dry_run;            /* 1: scheduling only, no device memory or kernels
                               (decode packets are then assumed innovative) */
    uint64_t budget_bytes;  /* device arena for request state and outputs */
} gf_serve_config;

typedef struct {
    uint64_t id;
    int kind;                /* 0 encode, 1 decode */
    int status;              /* GF_OK, or GF_ECANCELED (gf_serve_cancel) */
    int rank;                /* decode: N; encode: K */
    int packets_seen;        /* decode: packets taken into the echelon state */
    int packets_dropped;     /* decode: of those, not innovative */
    const uint8_t *out;      /* device: encode K rows / decode N rows */
    uint64_t ld_out;
    double t_submit, t_admit, t_done;
} gf_serve_done;

typedef struct {
    uint64_t steps, submitted, admitted, completed;
    uint64_t queued, active, inflight_steps;
    uint64_t arena_bytes, arena_used, arena_peak;
    uint64_t packets_pushed, packets_absorbed;
    uint64_t encode_tiles, absorb_items;
} gf_serve_counters;

int gf_serve_create(const gf_serve_config *cfg, gf_server **out);
void gf_serve_destroy(gf_server *sv);
/* C: device K x N; S: device N rows ld_s apart.  GF_ERANGE if the request
 * could never fit the arena. */
int gf_serve_submit_encode(gf_server *sv, uint64_t id, const uint8_t *C, int K, int N, const uint8_t *S,
                           size_t ld_s, size_t len, double now);
int gf_serve_submit_decode(gf_server *sv, uint64_t id, int N, size_t len, double now);
/* coef: device, N bytes; payload: device, len bytes. */
int gf_serve_push_packet(gf_server *sv, uint64_t id, const uint8_t *coef, const uint8_t *payload, double release);
/* The same for n packets at once: coef[i], payload[i], release[i] (host arrays). */
int gf_serve_push_packets(gf_server *sv, uint64_t id, int n, const uint8_t *const *coef,
                          const uint8_t *const *payload, const double *release);
/* Collect finished steps, admit, and enqueue one step.  Non-blocking unless
 * the in-flight window is full.  Returns the steps in flight (>= 0). */
int gf_serve_step(gf_server *sv, double now);
/* Up to `max` completed requests, oldest first; returns how many. */
int gf_serve_poll(gf_server *sv, gf_serve_done *out, int max);
/* Copy a polled request's output rows (K for encode, N for decode; len
 * bytes each) to dst (device, rows ld_dst apart).  The copy is enqueued on
 * `stream` (the caller's), after the caller's earlier work on it.  GF_EINVAL
 * for a cancelled request (it has no output). */
int gf_serve_copy_out(gf_server *sv, uint64_t id, uint8_t *dst, size_t ld_dst, void *stream);
/* Return a polled request's memory to the arena.  The memory is reused only
 * after no step in flight refers to it and every copy_out of the request has
 * run on its stream, so a release right after an (unfinished) copy_out is
 * safe. */
int gf_serve_release(gf_server *sv, uint64_t id);
/* What the server knows of a request that has not been released: its state
 * (0 queued, 1 admitted, 2 completed), the rank of a decode's echelon state as
 * of the last collected step (an encode: K once completed), the packets pushed
 * but not yet taken into a step, and the packets taken so far and dropped as
 * not innovative.  A sender uses it as the receiver's feedback.  GF_EINVAL for
 * an unknown or released id. */
typedef struct {
    int state;
    int rank;
    int packets_pending;
    int packets_seen;
    int packets_dropped;
} gf_serve_status;
int gf_serve_query(gf_server *sv, uint64_t id, gf_serve_status *out);

/* Give up on a request that has not completed, e.g. a decode whose sender
 * stopped before rank N.  A queued request completes at once; an admitted
 * decode takes no more packets and completes as soon as no step in flight
 * refers to it (a decode that reaches rank N in a step already in flight
 * completes normally).  It is then polled with status GF_ECANCELED and its
 * rank so far, has no output, and is released as usual.  GF_EINVAL for an
 * unknown, completed or already cancelled request, and for an admitted
 * encode (it completes in the step it is in). */
int gf_serve_cancel(gf_server *sv, uint64_t id, double now);
/* Wait for every step in flight and collect it. */
int gf_serve_drain(gf_server *sv, double now);
int gf_serve_stats(gf_server *sv, gf_serve_counters *out);

#ifdef __cplusplus
}
#endif
#endif
