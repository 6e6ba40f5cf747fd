// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

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
    uint32_t *ptab;   // [4][256][8]
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

// Per-generation descriptor as the persistent kernels read it.
struct DevGen {
    const uint8_t *C;
    const uint8_t *S;
    uint8_t *Y;
    uint64_t len, ld_s, ld_y;
    uint32_t K, N;
    const int *status;   // if non-null, the generation is skipped unless *status == need
    int need;
    uint32_t align;      // largest of 16, 8, 4, 1 dividing S, Y, ld_s and ld_y
};

// One wave tile of the persistent (table-form) encode: up to ENC_ROWS coded
// rows from k0, over `strips` consecutive strips of 256*d payload bytes from
// p0 (d dwords per lane), where D = d | (strips - 1) << 8; short generations
// take several strips per tile so that claims and descriptor loads amortise.
// The bit-matrix form uses gen and k0 only.
struct DevTile {
    uint32_t gen;
    uint16_t k0;
    uint16_t D;
    uint64_t p0;
};

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
    uint8_t *Csel;   // the innovative coefficient vectors as received, N x N (stride N)
    uint8_t *Cinv;   // Csel^-1 once the rank reaches N, N x N
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

#ifndef GF_MF_PREFETCH
#define GF_MF_PREFETCH 3
#endif
#ifndef GF_MF_WAVES_PER_SIMD
#define GF_MF_WAVES_PER_SIMD 2
#endif
constexpr int ENC_ROWS = GF_ENC_ROWS;   // coded rows per wave tile
inline uint64_t wave_strip(int D) { return 256ull * (uint64_t)D; }

hipError_t launch_region(int mode, uint8_t *y, const uint8_t *x, uint64_t len, const uint32_t *tab_host8,
                         hipStream_t s);
hipError_t launch_region_batched(const void *d_regions, int count, uint64_t max_len, const uint32_t *ptab_field,
                                 int q, hipStream_t s);
hipError_t launch_encode(int D, int nsplit, const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s,
                         uint8_t *Y, uint64_t ld_y, uint64_t len, const uint32_t *ptab_field, const int *status,
                         int need, bool aligned, hipStream_t s);
// Work queues of the persistent encode kernels.  Tiles sit in MF_QUEUES
// queues, one per XCD (workgroups are dealt to the 8 XCDs round robin, so
// workgroup b starts on queue b % 8 and moves on to the others when it is
// empty); all tiles of a generation share a queue, so its source stays in one
// L2.  A claim takes a run of consecutive tiles (short tiles are grouped, so
// claims stay rare).  runs[r] .. runs[r + 1] are the tiles of run r and
// bounds[i] .. bounds[i + 1] the runs of queue i.  Counter words, each on its
// own 256-byte line: MF_CTR_STRIDE * i, the next run of queue i;
// MF_CTR_RETIRED, the retired workgroups or waves.  The last to retire sets
// them all back to zero, so a launch needs no clearing beforehand.
constexpr int MF_QUEUES = 8;
constexpr int MF_CTR_STRIDE = 64;
constexpr int MF_CTR_RETIRED = MF_CTR_STRIDE * MF_QUEUES;
constexpr int GF_QUEUE_CTR_WORDS = MF_CTR_RETIRED + 1;

struct TileQueues {
    std::vector<DevTile> tiles;
    std::vector<unsigned> runs;      // number of runs + 1 entries
    unsigned bounds[MF_QUEUES + 1];
};
// Table form: wave tiles of ENC_ROWS coded rows x wave_strip(D) bytes.
void build_tiles(const DevGen *g, size_t n, int fixed_D, TileQueues &q);
// Bit-matrix form on the matrix cores: workgroup tiles of MF_ROWS coded rows
// over the whole packet length in strips of MF_STRIP bytes (DevTile.D unused).
constexpr int MF_ROWS = 16;
constexpr int MF_STRIP = 256;
void build_tiles_mfma(const DevGen *g, size_t n, TileQueues &q);

hipError_t launch_encode_persistent(const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                    const unsigned *bounds, int ntiles, unsigned *counters, int grid,
                                    const uint32_t *ptab_field, hipStream_t s);
// aligned4: every generation's source rows start 4-byte aligned.
hipError_t launch_encode_mfma(const DevGen *gens, const DevTile *tiles, const unsigned *runs, const unsigned *bounds,
                              int ntiles, unsigned *counters, int grid, const uint8_t *rows_field, bool aligned4,
                              hipStream_t s);
int encode_mfma_blocks_per_cu(bool aligned4);
// Bit-plane form (fields with n <= 4) over the table form's wave tiles.
hipError_t launch_encode_planes(int field, const DevGen *gens, const DevTile *tiles, const unsigned *runs,
                                const unsigned *bounds, int ntiles, unsigned *counters, int grid, hipStream_t s);
int encode_planes_blocks_per_cu(int field);
// One matrix (sys == nullptr: C, N, Cinv, rank) or `count` systems of one size
// class (N <= 32, 64, 128 or 256; N names the class), one workgroup each.
hipError_t launch_invert(const DevSys *sys, int count, const uint8_t *C, int N, uint8_t *Cinv, int *rank,
                         const uint32_t *ptab_field, const uint8_t *inv_field, hipStream_t s);
int encode_blocks_per_cu();
// One small generation in one launch (N, K <= 32, len <= 8192, rows 4-byte
// aligned: align from row_align): Y = C S, or for a decode (K = N) S = C^-1 B
// with the inversion in the same kernel, the rank written to *rank (if not
// null) and no output for a singular C.
bool small_ok(int K, int N, uint64_t len, uint32_t align);
hipError_t launch_small(const uint8_t *C, int K, int N, const uint8_t *S, uint64_t ld_s, uint8_t *Y, uint64_t ld_y,
                        uint64_t len, const uint32_t *ptab_field, const uint8_t *inv_field, int *rank, bool decode,
                        hipStream_t s);
uint32_t row_align(const void *S, uint64_t ld_s, const void *Y, uint64_t ld_y);
// Device tables of `field` on the current device (initialising it if needed).
int gfnc_field_tables(int field, const uint32_t **ptab, const uint8_t **inv);
const uint8_t *gfnc_field_rows(int field);
hipError_t launch_absorb(const DevAbsorb *items, int n, const DevPacket *pkts, const uint32_t *ptab_field,
                         const uint8_t *inv_field, hipStream_t s);
hipError_t launch_meta_init(int *const *metas, int n, hipStream_t s);
hipError_t launch_status_gather(int *const *metas, int n, int4 *out, hipStream_t s);

}  // namespace gfnc
