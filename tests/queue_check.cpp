// Host check of the persistent encode kernels' work queues (no GPU needed):
// builds the queues of random batches with the library's own builders and
// checks their invariants.  Exit status 0 when every check holds.
//
//   * runs partition the tile list in order; queue bounds partition the runs;
//   * bit-matrix form: every (generation, 16-row block) of a generation with
//     rows and payload appears exactly once, nothing else appears;
//   * table form: for every generation and 24-row block the tiles' strips
//     cover [0, len) exactly once, in order, with the declared lane widths;
//   * all tiles of one generation sit in one queue;
//   * small-generation streaming form (queued) and its chunked form (one wave
//     per tile, no queues): every generation's strips of 1 KiB covered once,
//     in order, within the per-tile strip limit; the chunked runs of a
//     generation differ in length by at most one strip.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "gf_internal.h"

using namespace gfnc;

static int failures = 0;
#define CHECK(cond, ...)                                                                                          \
    do {                                                                                                          \
        if (!(cond)) {                                                                                            \
            std::fprintf(stderr, __VA_ARGS__);                                                                    \
            std::fprintf(stderr, "\n");                                                                           \
            if (++failures > 20)                                                                                  \
                std::exit(1);                                                                                     \
        }                                                                                                         \
    } while (0)

static void check_structure(const TileQueues &q, size_t ngen, const char *what)
{
    CHECK(!q.runs.empty() && q.runs.front() == 0, "%s: runs must start at tile 0", what);
    CHECK(q.runs.back() == q.tiles.size(), "%s: runs must end at the tile count", what);
    for (size_t r = 0; r + 1 < q.runs.size(); r++)
        CHECK(q.runs[r] < q.runs[r + 1], "%s: run %zu is empty or out of order", what, r);
    CHECK(q.bounds[0] == 0, "%s: queue 0 must start at run 0", what);
    for (int i = 0; i < MF_QUEUES; i++)
        CHECK(q.bounds[i] <= q.bounds[i + 1], "%s: queue bounds out of order", what);
    CHECK(q.bounds[MF_QUEUES] + 1 == q.runs.size(), "%s: queues must cover every run", what);
    // the queue of each tile, and one queue per generation
    std::map<uint32_t, int> queue_of;
    for (int i = 0; i < MF_QUEUES; i++)
        for (unsigned r = q.bounds[i]; r < q.bounds[i + 1]; r++)
            for (unsigned t = q.runs[r]; t < q.runs[r + 1]; t++) {
                const uint32_t g = q.tiles[t].gen;
                CHECK(g < ngen, "%s: tile %u names generation %u of %zu", what, t, g, ngen);
                auto it = queue_of.find(g);
                if (it == queue_of.end())
                    queue_of[g] = i;
                else
                    CHECK(it->second == i, "%s: generation %u spans queues %d and %d", what, g, it->second, i);
            }
}

// Strips [p0, p0 + strips * 1 KiB) of each generation must cover [0, len)
// once, in order, and every strip must start inside the row.
static void check_strip_cover(const std::vector<DevTile> &tiles, const std::vector<DevGen> &g, int max_strips,
                              bool equal_runs, const char *what)
{
    std::map<uint32_t, std::vector<std::pair<uint64_t, int>>> cover;
    for (const DevTile &t : tiles) {
        const int strips = (t.D >> 8) + 1;
        CHECK((t.D & 0xFF) == 4, "%s: lane width %d", what, t.D & 0xFF);
        CHECK(t.k0 == 0, "%s: tile starts at row %u", what, t.k0);
        CHECK(strips <= max_strips, "%s: %d strips in a tile, at most %d", what, strips, max_strips);
        CHECK(t.gen < g.size(), "%s: tile names generation %u of %zu", what, t.gen, g.size());
        if (t.gen < g.size())
            cover[t.gen].push_back({t.p0, strips});
    }
    for (size_t i = 0; i < g.size(); i++) {
        auto it = cover.find((uint32_t)i);
        if (!g[i].K || !g[i].len) {
            CHECK(it == cover.end(), "%s: generation %zu has no work but has tiles", what, i);
            continue;
        }
        CHECK(it != cover.end(), "%s: generation %zu not covered", what, i);
        if (it == cover.end())
            continue;
        const auto &v = it->second;   // in the builders' order, which must be the row order
        uint64_t at = 0;
        int lo = 1 << 30, hi = 0;
        for (const auto &s : v) {
            CHECK(s.first == at, "%s: gen %zu gap, overlap or disorder at %llu", what, i, (unsigned long long)at);
            CHECK(s.first < g[i].len, "%s: gen %zu has a tile past the end", what, i);
            at = s.first + 1024ull * (uint64_t)s.second;
            lo = std::min(lo, s.second);
            hi = std::max(hi, s.second);
        }
        CHECK(at >= g[i].len && at < g[i].len + 1024, "%s: gen %zu ends at %llu for %llu bytes", what, i,
              (unsigned long long)at, (unsigned long long)g[i].len);
        if (equal_runs)
            CHECK(hi - lo <= 1, "%s: gen %zu runs of %d to %d strips", what, i, lo, hi);
    }
}

int main()
{
    std::mt19937_64 rng(190902871);
    for (int trial = 0; trial < 40; trial++) {
        const size_t n = 1 + rng() % 400;
        std::vector<DevGen> g(n);
        for (size_t i = 0; i < n; i++) {
            DevGen &x = g[i];
            x = DevGen{};
            x.K = (rng() % 10 == 0) ? 0 : 1 + (uint32_t)(rng() % 300);
            x.N = 1 + (uint32_t)(rng() % 256);
            const int shape = (int)(rng() % 10);
            x.len = shape == 0 ? 0 : shape == 1 ? 1 + rng() % 300 : 64 + rng() % 20000;
            x.ld_s = x.ld_y = x.len;
        }
        // bit-matrix form
        {
            TileQueues q;
            build_tiles_mfma(g.data(), n, q);
            check_structure(q, n, "mfma");
            std::set<std::pair<uint32_t, uint32_t>> seen;
            for (const DevTile &t : q.tiles) {
                CHECK(t.k0 % MF_ROWS == 0 && t.k0 < g[t.gen].K, "mfma: bad k0 %u for K %u", t.k0, g[t.gen].K);
                CHECK(seen.insert({t.gen, t.k0}).second, "mfma: tile (%u, %u) twice", t.gen, t.k0);
            }
            size_t want = 0;
            for (size_t i = 0; i < n; i++)
                if (g[i].K && g[i].len)
                    want += (g[i].K + MF_ROWS - 1) / MF_ROWS;
            CHECK(seen.size() == want, "mfma: %zu tiles, want %zu", seen.size(), want);
        }
        // table form, each lane width choice
        for (int fixed_D : {0, 1, 2, 4}) {
            TileQueues q;
            build_tiles(g.data(), n, fixed_D, q);
            check_structure(q, n, "table");
            std::map<std::pair<uint32_t, uint32_t>, std::vector<std::pair<uint64_t, uint64_t>>> cover;
            for (const DevTile &t : q.tiles) {
                const int d = t.D & 0xFF, strips = (t.D >> 8) + 1;
                CHECK(d == 1 || d == 2 || d == 4, "table: lane width %d", d);
                CHECK(fixed_D == 0 || d == fixed_D, "table: width %d, forced %d", d, fixed_D);
                CHECK(t.k0 % ENC_ROWS == 0 && t.k0 < g[t.gen].K, "table: bad k0 %u", t.k0);
                cover[{t.gen, t.k0}].push_back({t.p0, t.p0 + (uint64_t)strips * wave_strip(d)});
            }
            for (size_t i = 0; i < n; i++) {
                if (!g[i].K || !g[i].len)
                    continue;
                for (uint32_t k0 = 0; k0 < g[i].K; k0 += ENC_ROWS) {
                    auto it = cover.find({(uint32_t)i, k0});
                    CHECK(it != cover.end(), "table: generation %zu rows %u not covered", i, k0);
                    if (it == cover.end())
                        continue;
                    auto v = it->second;
                    std::sort(v.begin(), v.end());
                    uint64_t at = 0;
                    for (auto &s : v) {
                        CHECK(s.first == at, "table: gen %zu rows %u gap or overlap at %llu", i, k0,
                              (unsigned long long)at);
                        at = s.second;
                    }
                    CHECK(at >= g[i].len, "table: gen %zu rows %u ends at %llu < %llu", i, k0,
                          (unsigned long long)at, (unsigned long long)g[i].len);
                    CHECK(v.back().first < g[i].len, "table: gen %zu rows %u has a tile past the end", i, k0);
                }
            }
        }
        // small-generation streaming form, queued and chunked
        {
            std::vector<DevGen> sg = g;
            for (DevGen &x : sg) {
                x.K = x.K ? 1 + x.K % STREAM_MAX : 0;
                x.N = 1 + x.N % STREAM_MAX;
                if (rng() % 8 == 0)
                    x.len = 1024 * (1 + rng() % 200) + rng() % 3;   // lengths near whole strips
            }
            TileQueues q;
            build_tiles_stream(sg.data(), n, q);
            check_structure(q, n, "stream");
            check_strip_cover(q.tiles, sg, STREAM_STRIPS, false, "stream");
            for (int sk : {1, 2, 4, 8}) {
                const int burst = encode_chunks_strips(sk);
                CHECK(burst >= 1, "chunks: %d strips per tile for K %d", burst, sk);
                std::vector<DevTile> tiles;
                build_tiles_chunks(sg.data(), n, burst, tiles);
                check_strip_cover(tiles, sg, burst, true, "chunks");
                for (size_t t = 1; t < tiles.size(); t++)
                    CHECK(tiles[t - 1].gen <= tiles[t].gen, "chunks: tiles out of generation order at %zu", t);
            }
        }
    }
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("queue checks ok\n");
    return 0;
}
