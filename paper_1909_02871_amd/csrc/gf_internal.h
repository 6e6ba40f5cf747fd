// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gf_types.h"

namespace gfnc {

// Field index 0..3 for n = 1, 2, 4, 8.
inline int field_index(int n) { return n == 1 ? 0 : n == 2 ? 1 : n == 4 ? 2 : n == 8 ? 3 : -1; }

// Device-resident tables for one device.
//   ptab[f][c][0..7]: byte-permute product tables of coefficient c in field f
//     dwords 0,1: c * v for the 8 bytes v whose set bits lie in bits 0-2
//     dwords 2,3: c * (v << 3), v < 8
//     dword  4  : c * (v << 6), v < 4
//     dwords 5-7: zero
//     (c * b is applied word by word, so every field shares one kernel; rows
//      with c >= q are all zero.)
//   inv[f][a]: multiplicative inverse of a (0 for a = 0 or a >= q).
//   rows[f][c][i]: row i of the 8 x 8 bit matrix of "multiply a byte by c":
//     bit j is bit i of c * (1 << j)  (the product is GF(2)-linear in the byte).
struct DevTables {
    uint32_t *ptab;   // [8][256][8]: [f] the product tables, [4 + f] those of c's inverse at c
    uint8_t *inv;     // [4][256]
    uint8_t *rows;    // [4][256][8]
};

// Host copies, built once by build_tables().
struct HostTables {
    uint32_t ptab[4][256][8];
    uint8_t inv[4][256];
    uint8_t mul[4][256][256];   // element products (row c, column a), a, c < q
    uint8_t rows[4][256][8];    // bit-matrix rows, as in DevTables
};
const HostTables &host_tables();

struct DevSys {
    const uint8_t *C;
    uint8_t *Cinv;
    int *rank;
    uint32_t N;
    uint32_t pad;
};

#ifndef GF_ENC_ROWS
#define GF_ENC_ROWS 24
#endif
#ifndef GF_ENC_WAVES_PER_SIMD
#define GF_ENC_WAVES_PER_SIMD 2
#endif
#ifndef GF_PLANE_WAVES_PER_SIMD
#define GF_PLANE_WAVES_PER_SIMD 3   // bit-plane form, n <= 2 (n = 4 needs the registers of 2)
#endif
// Device state of one generation being decoded progressively (serving).
struct DevDecSlot {
    uint8_t *R;      // reduced echelon rows of the innovative coefficient vectors, row stride rs
    uint8_t *T;      // R = T Csel: weights of the accepted packets in each row of R, row stride rs
    uint8_t *Cinv;   // Csel^-1 once the rank reaches N, N x N (Csel: the accepted vectors as received)
    uint8_t *Bsel;   // payloads of the innovative packets, row i at Bsel + i*ld
    int *meta;       // [0] rank, [1] step that completed it (-1 before), [2] packets seen,
                     // [3] packets that were not innovative, [4 .. 4+N) pivot column of row i
    uint64_t len, ld;
    uint32_t N, rs;
};

struct DevAbsorb {
    DevDecSlot s;
    uint32_t pk0, npk;   // packets [pk0, pk0 + npk) of the step's packet list
    int step;
    int pad;
};

struct DevPacket {
    const uint8_t *coef;      // N coefficients
    const uint8_t *payload;   // len bytes
};

// Tables of a batched decode that its descriptors are read into on the device
// (all inside the caller's workspace): see k_dec_schedule.
struct DecSched {
    unsigned *cls_count;   // [4] systems per elimination size class
    unsigned *bounds;      // [2][MF_QUEUES + 1] queue bounds of the two product kernels
    unsigned *ctr;         // [2][GF_QUEUE_CTR_WORDS] their queue counters
    DevSys *lists;         // [4][count] systems of each size class
    DevGen *gens;          // [count] product S = C^-1 B of each system
    DevTile *tiles;        // [2][tile_cap] tiles of each product kernel
    uint64_t tile_cap;
    int *rank;             // [count]
    uint8_t *inv;          // [count][slot] inverses
    uint64_t slot;
};

// The autotuner's choice for a class of batches (gf_tune.cpp): kernel form,
// dwords per lane (0: per tile), share of the full persistent grid in percent,
// and the measured milliseconds.
struct TuneChoice {
    int form, fixed_D, grid_pct;
    double ms;
};
std::string tune_key(int field, const std::vector<DevGen> &g, bool aligned4, int req_form, int req_bpl,
                     int req_grid);
bool tune_cache_get(const std::string &key, TuneChoice *out);
void tune_cache_put(const std::string &key, const TuneChoice &c);

constexpr int ENC_ROWS = GF_ENC_ROWS;   // coded rows per wave tile
inline uint64_t wave_strip(int D) { return 256ull * (uint64_t)D; }

hipError_t launch_region(int mode, uint8_t *y, const uint8_t *x, uint64_t len, const uint32_t *tab_host8,
                         hipStream_t s);
hipError_t launch_region_batched(const void *d_regions, int count, uint64_t max_len, const uint32_t *ptab_field,
                                 int q, hipStream_t s);
hipError_t launch_encode(int D, int nsplit, const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s,
                         uint8_t *Y, uint64_t ld_y, uint64_t len, const uint32_t *ptab_field, const int *status,
                         int need, bool aligned, hipStream_t s);

struct TileQueues {
    std::vector<DevTile> tiles;
    std::vector<unsigned> runs;      // number of runs + 1 entries
    unsigned bounds[MF_QUEUES + 1];
};
// Table form: wave tiles of ENC_ROWS coded rows x wave_strip(D) bytes.
void build_tiles(const DevGen *g, size_t n, int fixed_D, TileQueues &q);
// Bit-matrix form on the matrix cores: workgroup tiles of MF_ROWS coded rows
// over the whole packet length in strips of MF_STRIP bytes (DevTile.D unused).
void build_tiles_mfma(const DevGen *g, size_t n, TileQueues &q);

// direct: not persistent, a workgroup per four wave tiles (grid unused).
hipError_t launch_encode_persistent(const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                    const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                    const uint32_t *ptab_field, hipStream_t s, bool direct = false);
// aligned4: every generation's source rows start 4-byte aligned.
hipError_t launch_encode_mfma(const DevGen *gens, const DevTile *tiles, const unsigned *runs, const unsigned *bounds,
                              int ntiles, unsigned *counters, int grid, const uint8_t *rows_field, bool aligned4,
                              hipStream_t s);
int encode_mfma_blocks_per_cu(bool aligned4);
// Bit-plane form (fields with n <= 4) over the table form's wave tiles.
hipError_t launch_encode_planes(int field, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid, hipStream_t s,
                                bool direct = false);
int encode_planes_blocks_per_cu(int field);
// Small-generation streaming form (every generation K <= 8 and N <= 8): wave
// tiles of up to STREAM_STRIPS strips of 1 KiB, tables staged once per tile.
constexpr int STREAM_MAX = 8;
constexpr int STREAM_STRIPS = 64;
void build_tiles_stream(const DevGen *g, size_t n, TileQueues &q);
// sk: the batch's largest K or N (the kernel is instantiated for 1, 2, 4 and 8).
hipError_t launch_encode_stream(int sk, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                const uint32_t *ptab_field, hipStream_t s);
int encode_stream_blocks_per_cu(int sk);
// The same generations without queues: one wave per tile of at most
// encode_chunks_strips(sk) strips, a workgroup per four tiles.
int encode_chunks_strips(int sk);
void build_tiles_chunks(const DevGen *g, size_t n, int burst, std::vector<DevTile> &tiles);
hipError_t launch_encode_chunks(int sk, const DevGen *gens, const DevTile *tiles, int ntiles,
                                const uint32_t *ptab_field, hipStream_t s);
// One matrix (sys == nullptr: C, N, Cinv, rank) or `count` systems of one size
// class (N <= 32, 64, 128 or 256; N names the class), one workgroup each.
hipError_t launch_invert(const DevSys *sys, int count, const uint8_t *C, int N, uint8_t *Cinv, int *rank,
                         const uint32_t *ptab_field, const uint8_t *inv_field, hipStream_t s,
                         const unsigned *d_count = nullptr);
// Device-side set-up of the descriptor-driven batched calls (gf_sched.hip).
hipError_t launch_bind_gens(const void *d_ext, const DevGen *shape, DevGen *out, int count, unsigned *err,
                            const int *skip, hipStream_t s);
hipError_t launch_dec_schedule(const void *d_sys, int count, const DecSched &w, hipStream_t s);
int encode_blocks_per_cu();
// One small generation in one launch (N, K <= 32, len <= 8192, rows 4-byte
// aligned: align from row_align): Y = C S, or for a decode (K = N) S = C^-1 B
// with the inversion in the same kernel, the rank written to *rank (if not
// null) and no output for a singular C.
bool small_ok(int K, int N, uint64_t len, uint32_t align);
hipError_t launch_small(const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s, uint8_t *Y, uint64_t ld_y,
                        uint64_t len, const uint32_t *ptab_field, const uint32_t *ptab_inv_field,
                        const uint8_t *inv_field, int *rank, bool decode,
                        hipStream_t s);
uint32_t row_align(const void *S, uint64_t ld_s, const void *Y, uint64_t ld_y);
// Device tables of `field` on the current device (initialising it if needed).
int gfnc_field_tables(int field, const uint32_t **ptab, const uint8_t **inv);
const uint8_t *gfnc_field_rows(int field);
// Instruction-mix microbenchmarks (gf_ceiling.hip): 0 device copy, 1 table
// step, 2 FP4 MFMA, 3 bit-plane step.
hipError_t launch_ceiling(int what, void *buf, uint64_t bytes, int blocks, int iters, hipStream_t s);
hipError_t launch_absorb(const DevAbsorb *items, int n, const DevPacket *pkts, const uint32_t *ptab_field,
                         const uint8_t *inv_field, hipStream_t s);
hipError_t launch_meta_init(int *const *metas, int n, hipStream_t s);
hipError_t launch_status_gather(int *const *metas, int n, int4 *out, hipStream_t s);

}  // namespace gfnc
