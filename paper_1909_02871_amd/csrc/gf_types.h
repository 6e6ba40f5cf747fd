// Types and constants that the persistent encode kernels share with the host
// code that builds their schedules (kept apart from the host-only declarations
// so that a kernel's sources change only when something it uses does).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef GF_MF_PREFETCH
#define GF_MF_PREFETCH 3
#endif
#ifndef GF_MF_WAVES_PER_SIMD
#define GF_MF_WAVES_PER_SIMD 2
#endif

namespace gfnc {

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

// Bit-matrix form on the matrix cores: workgroup tiles of MF_ROWS coded rows
// over the whole packet length in strips of MF_STRIP bytes (DevTile.D unused).
constexpr int MF_ROWS = 16;
constexpr int MF_STRIP = 256;

}  // namespace gfnc
