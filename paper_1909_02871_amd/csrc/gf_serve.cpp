// Serving runtime: continuous batching of encode and progressive-decode
// requests over one device arena.
//
// A step (gf_serve_step) admits queued requests in FIFO order while a slot
// and arena memory are free, then enqueues, on the server's stream, one
// absorb launch (every decode generation with packets released by `now`
// takes up to `burst` of them into its device-resident echelon state), one
// persistent encode launch (all newly admitted encode requests plus the
// payload product of every decode generation that the absorb launch may
// complete), and a status read-back.  Up to kInflight steps are in flight;
// results are collected in order, so requests arriving while others run join
// the next step.  Each request's bytes depend only on its own inputs: steps
// never combine generations arithmetically.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/gfnc.h"
#include "gf_internal.h"

using namespace gfnc;

namespace {

constexpr int kInflight = 2;
constexpr uint64_t kAlign = 256;

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing; bookkeeping only.
class Arena {
  public:
    explicit Arena(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        n = round_up(std::max<uint64_t>(n, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const uint64_t o = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest)
                    free_[o + n] = rest;
                *off = o;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = round_up(std::max<uint64_t>(n, 1), kAlign);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_, used_ = 0, peak_ = 0;
};

enum { QUEUED = 0, ACTIVE = 1, DONE = 2 };

struct Packet {
    const uint8_t *coef, *payload;
    double release;
};

struct Req {
    uint64_t id = 0;
    int kind = 0;   // 0 encode, 1 decode
    int N = 0, K = 0;
    uint64_t len = 0, ld = 0;
    const uint8_t *C = nullptr, *S = nullptr;
    uint64_t ld_s = 0;
    int state = QUEUED;
    int status = GF_OK;       // GF_ECANCELED once cancelled
    bool launched = false, polled = false, release_asked = false, cancel = false;
    std::vector<hipEvent_t> copies;   // recorded after each copy_out on the caller's stream
    uint64_t off = 0, bytes = 0;
    uint8_t *out = nullptr;
    DevDecSlot slot{};
    std::deque<Packet> pkts;
    int rank = 0, seen = 0, dropped = 0;
    int64_t last_step = -1;   // last step whose kernels reference the request's memory
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct StepBuf {
    char *host = nullptr, *dev = nullptr;
    size_t cap = 0;
    int4 *d_status = nullptr, *h_status = nullptr;
    size_t status_cap = 0;
    hipEvent_t ev = nullptr;
};

struct InFlight {
    int64_t step;
    int buf;
    std::vector<Req *> enc, dec;
};

}  // namespace

struct gf_server {
    gf_serve_config cfg{};
    std::mutex mu;
    Arena arena{0};
    uint8_t *base = nullptr;
    hipStream_t stream = nullptr;
    unsigned *ctr = nullptr;
    const uint32_t *ptab = nullptr;
    const uint8_t *inv = nullptr;
    const uint8_t *rows = nullptr;   // bit-matrix rows of the field
    int grid_max = 1;                // table-form workgroups at once
    int grid_max_mf = 1;             // bit-matrix workgroups at once
    int64_t next_step = 0;
    std::unordered_map<uint64_t, Req *> reqs;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::deque<Req *> done_fifo;
    std::vector<Req *> to_free;
    std::deque<InFlight> inflight;
    StepBuf bufs[kInflight + 1];
    int next_buf = 0;
    gf_serve_counters st{};
    int err = GF_OK;   // first device or memory failure of a step; sticky
};

namespace {

uint64_t footprint(const Req &r)
{
    if (r.kind == 0)
        return round_up((uint64_t)r.K * r.ld, kAlign);
    const uint64_t N = (uint64_t)r.N, rs = round_up(N, 4);
    return 2 * round_up(N * rs, kAlign) + round_up(N * N, kAlign) + 2 * round_up(N * r.ld, kAlign) +
           round_up((4 + N) * sizeof(int), kAlign);
}

void layout(gf_server *sv, Req &r)
{
    uint8_t *p = sv->base + r.off;
    if (r.kind == 0) {
        r.out = p;
        return;
    }
    const uint64_t N = (uint64_t)r.N, rs = round_up(N, 4);
    DevDecSlot &s = r.slot;
    s.R = p;
    p += round_up(N * rs, kAlign);
    s.T = p;
    p += round_up(N * rs, kAlign);
    s.Cinv = p;
    p += round_up(N * N, kAlign);
    s.Bsel = p;
    p += round_up(N * r.ld, kAlign);
    r.out = p;
    p += round_up(N * r.ld, kAlign);
    s.meta = reinterpret_cast<int *>(p);
    s.len = r.len;
    s.ld = r.ld;
    s.N = (uint32_t)r.N;
    s.rs = (uint32_t)rs;
}

// True once every copy_out of the request (on the callers' streams) has run.
bool copies_done(Req *r)
{
    while (!r->copies.empty()) {
        const hipError_t q = hipEventQuery(r->copies.back());
        if (q == hipErrorNotReady)
            return false;
        (void)hipEventDestroy(r->copies.back());   // finished (or failed: nothing left to wait for)
        r->copies.pop_back();
    }
    return true;
}

// Return released requests' memory once no step in flight refers to it and
// their copies out have completed, so a later request can never overwrite
// bytes a copy still reads.
void free_ready(gf_server *sv, int64_t completed_step)
{
    std::vector<Req *> keep;
    for (Req *r : sv->to_free) {
        if (r->last_step <= completed_step && copies_done(r)) {
            if (r->bytes)
                sv->arena.release(r->off, r->bytes);
            sv->reqs.erase(r->id);
            delete r;
        } else {
            keep.push_back(r);
        }
    }
    sv->to_free.swap(keep);
}

// The last step whose kernels have all completed.
int64_t retired_step(const gf_server *sv)
{
    return sv->inflight.empty() ? sv->next_step - 1 : sv->inflight.front().step - 1;
}

void finish(gf_server *sv, Req *r, double now, int status = GF_OK)
{
    if (r->state == DONE)
        return;
    r->state = DONE;
    r->status = status;
    r->t_done = now;
    sv->active.erase(std::remove(sv->active.begin(), sv->active.end(), r), sv->active.end());
    sv->done_fifo.push_back(r);
    sv->st.completed++;
}

// Results of the oldest in-flight step (the caller knows it has finished).
void retire(gf_server *sv, double now)
{
    InFlight f = sv->inflight.front();
    sv->inflight.pop_front();
    const StepBuf &b = sv->bufs[f.buf];
    for (Req *r : f.enc)
        finish(sv, r, now);
    for (size_t i = 0; i < f.dec.size(); i++) {
        Req *r = f.dec[i];
        int rank, done_step, seen, dropped;
        if (sv->cfg.dry_run) {
            rank = r->rank;
            done_step = rank >= r->N ? (int)f.step : -1;
            seen = r->seen;
            dropped = r->dropped;
        } else {
            const int4 v = b.h_status[i];
            rank = v.x;
            done_step = v.y;
            seen = v.z;
            dropped = v.w;
        }
        r->rank = rank;
        r->seen = seen;
        r->dropped = dropped;
        if (done_step >= 0)
            finish(sv, r, now);
        else if (r->cancel && r->last_step <= f.step)
            finish(sv, r, now, GF_ECANCELED);
    }
    free_ready(sv, f.step);
}

int collect(gf_server *sv, double now, bool block_until_room)
{
    while (!sv->inflight.empty()) {
        const StepBuf &b = sv->bufs[sv->inflight.front().buf];
        bool ready = true;
        if (!sv->cfg.dry_run) {
            const bool must = block_until_room && (int)sv->inflight.size() >= kInflight;
            if (must) {
                if (hipEventSynchronize(b.ev) != hipSuccess)
                    return GF_EDEVICE;
            } else {
                const hipError_t q = hipEventQuery(b.ev);
                if (q == hipErrorNotReady)
                    ready = false;
                else if (q != hipSuccess)
                    return GF_EDEVICE;
            }
        }
        if (!ready)
            break;
        retire(sv, now);
    }
    return GF_OK;
}

int ensure_buf(StepBuf &b, size_t bytes, size_t nstatus)
{
    if (bytes > b.cap) {
        if (b.host)
            (void)hipHostFree(b.host);
        if (b.dev)
            (void)hipFree(b.dev);
        b.host = nullptr;
        b.dev = nullptr;
        const size_t cap = std::max<size_t>(bytes * 2, 1 << 20);
        if (hipHostMalloc(reinterpret_cast<void **>(&b.host), cap, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b.dev), cap) != hipSuccess)
            return GF_ENOMEM;
        b.cap = cap;
    }
    if (nstatus > b.status_cap) {
        if (b.h_status)
            (void)hipHostFree(b.h_status);
        if (b.d_status)
            (void)hipFree(b.d_status);
        b.h_status = nullptr;
        b.d_status = nullptr;
        const size_t cap = std::max<size_t>(nstatus * 2, 1024);
        if (hipHostMalloc(reinterpret_cast<void **>(&b.h_status), cap * sizeof(int4), hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b.d_status), cap * sizeof(int4)) != hipSuccess)
            return GF_ENOMEM;
        b.status_cap = cap;
    }
    return GF_OK;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// A step or drain that fails part-way leaves requests taken off their queues
// but never launched or collected, so the server refuses further work.
int fail(gf_server *sv, int rc)
{
    if (rc && !sv->err)
        sv->err = rc;
    return rc;
}

}  // namespace

extern "C" {

int gf_serve_create(const gf_serve_config *cfg, gf_server **out)
{
    if (!out)
        return GF_EINVAL;
    *out = nullptr;
    if (!cfg || (cfg->field != 1 && cfg->field != 2 && cfg->field != 4 && cfg->field != 8) || cfg->max_slots < 0 ||
        cfg->burst < 0 || cfg->budget_bytes < kAlign)
        return GF_EINVAL;
    gf_server *sv = new (std::nothrow) gf_server;
    if (!sv)
        return GF_ENOMEM;
    sv->cfg = *cfg;
    if (sv->cfg.max_slots == 0)
        sv->cfg.max_slots = 1024;
    if (sv->cfg.burst == 0)
        sv->cfg.burst = 64;
    sv->arena = Arena(cfg->budget_bytes);
    if (cfg->dry_run) {
        sv->base = reinterpret_cast<uint8_t *>((uintptr_t)1 << 40);   // never dereferenced
        *out = sv;
        return GF_OK;
    }
    int rc = gf_init();
    if (rc) {
        delete sv;
        return rc;
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    sv->grid_max = std::max(1, cus) * encode_blocks_per_cu();
    sv->grid_max_mf = std::max(1, cus) * encode_mfma_blocks_per_cu(true);
    const HostTables &h = host_tables();
    (void)h;
    if (hipMalloc(reinterpret_cast<void **>(&sv->base), cfg->budget_bytes) != hipSuccess) {
        delete sv;
        return GF_ENOMEM;
    }
    if (hipMalloc(reinterpret_cast<void **>(&sv->ctr), GF_QUEUE_CTR_WORDS * sizeof(unsigned)) != hipSuccess ||
        hipMemset(sv->ctr, 0, GF_QUEUE_CTR_WORDS * sizeof(unsigned)) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
        gf_serve_destroy(sv);
        return GF_EDEVICE;
    }
    for (StepBuf &b : sv->bufs)
        if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
            gf_serve_destroy(sv);
            return GF_EDEVICE;
        }
    rc = gfnc_field_tables(cfg->field, &sv->ptab, &sv->inv);
    if (rc) {
        gf_serve_destroy(sv);
        return rc;
    }
    sv->rows = gfnc_field_rows(cfg->field);
    *out = sv;
    return GF_OK;
}

void gf_serve_destroy(gf_server *sv)
{
    if (!sv)
        return;
    if (!sv->cfg.dry_run) {
        if (sv->stream)
            (void)hipStreamSynchronize(sv->stream);
        for (auto &kv : sv->reqs)   // copies out still reading the arena
            for (hipEvent_t ev : kv.second->copies)
                (void)hipEventSynchronize(ev);
        for (StepBuf &b : sv->bufs) {
            if (b.host)
                (void)hipHostFree(b.host);
            if (b.dev)
                (void)hipFree(b.dev);
            if (b.h_status)
                (void)hipHostFree(b.h_status);
            if (b.d_status)
                (void)hipFree(b.d_status);
            if (b.ev)
                (void)hipEventDestroy(b.ev);
        }
        if (sv->stream)
            (void)hipStreamDestroy(sv->stream);
        (void)hipFree(sv->ctr);
        (void)hipFree(sv->base);
    }
    for (auto &kv : sv->reqs) {
        for (hipEvent_t ev : kv.second->copies)
            (void)hipEventDestroy(ev);
        delete kv.second;
    }
    delete sv;
}

int gf_serve_submit_encode(gf_server *sv, uint64_t id, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s,
                           size_t len, double now)
{
    if (!sv || K < 1 || N < 1 || len == 0 || !C || !S || (N > 1 && ld_s < len))
        return GF_EINVAL;
    if (N > GF_MAX_N || K > GF_MAX_K)
        return GF_ERANGE;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err)
        return sv->err;
    if (sv->reqs.count(id))
        return GF_EINVAL;
    Req *r = new Req;
    r->id = id;
    r->kind = 0;
    r->N = N;
    r->K = K;
    r->len = len;
    r->ld = round_up(len, 16);
    r->C = C;
    r->S = S;
    r->ld_s = ld_s;
    r->t_submit = now;
    r->bytes = footprint(*r);
    if (r->bytes > sv->arena.size()) {
        delete r;
        return GF_ERANGE;
    }
    sv->reqs[id] = r;
    sv->queue.push_back(r);
    sv->st.submitted++;
    return GF_OK;
}

int gf_serve_submit_decode(gf_server *sv, uint64_t id, int N, size_t len, double now)
{
    if (!sv || N < 1 || len == 0)
        return GF_EINVAL;
    if (N > GF_MAX_N)
        return GF_ERANGE;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err)
        return sv->err;
    if (sv->reqs.count(id))
        return GF_EINVAL;
    Req *r = new Req;
    r->id = id;
    r->kind = 1;
    r->N = N;
    r->K = N;
    r->len = len;
    r->ld = round_up(len, 16);
    r->t_submit = now;
    r->bytes = footprint(*r);
    if (r->bytes > sv->arena.size()) {
        delete r;
        return GF_ERANGE;
    }
    sv->reqs[id] = r;
    sv->queue.push_back(r);
    sv->st.submitted++;
    return GF_OK;
}

int gf_serve_push_packet(gf_server *sv, uint64_t id, const uint8_t *coef, const uint8_t *payload, double release)
{
    if (!sv || !coef || !payload)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err)
        return sv->err;
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end() || it->second->kind != 1 || it->second->state == DONE || it->second->cancel)
        return GF_EINVAL;
    Req *r = it->second;
    // keep the queue ordered by release time (stable for equal times)
    auto pos = r->pkts.end();
    while (pos != r->pkts.begin() && std::prev(pos)->release > release)
        --pos;
    r->pkts.insert(pos, Packet{coef, payload, release});
    sv->st.packets_pushed++;
    return GF_OK;
}

int gf_serve_push_packets(gf_server *sv, uint64_t id, int n, const uint8_t *const *coef,
                          const uint8_t *const *payload, const double *release)
{
    if (!sv || n < 0 || (n > 0 && (!coef || !payload || !release)))
        return GF_EINVAL;
    for (int i = 0; i < n; i++)
        if (!coef[i] || !payload[i])
            return GF_EINVAL;
    for (int i = 0; i < n; i++) {
        const int rc = gf_serve_push_packet(sv, id, coef[i], payload[i], release[i]);
        if (rc)
            return rc;
    }
    return GF_OK;
}

int gf_serve_step(gf_server *sv, double now)
{
    if (!sv)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err)
        return sv->err;
    int rc = collect(sv, now, true);
    if (rc)
        return fail(sv, rc);
    free_ready(sv, retired_step(sv));

    // admission: FIFO, stop at the first request that does not fit
    std::vector<Req *> admitted;
    while (!sv->queue.empty() && (int)sv->active.size() < sv->cfg.max_slots) {
        Req *r = sv->queue.front();
        uint64_t off;
        if (!sv->arena.alloc(r->bytes, &off))
            break;
        sv->queue.pop_front();
        r->off = off;
        layout(sv, *r);
        r->state = ACTIVE;
        r->t_admit = now;
        sv->active.push_back(r);
        admitted.push_back(r);
        sv->st.admitted++;
    }

    const int64_t step = sv->next_step;
    InFlight f{step, sv->next_buf, {}, {}};
    std::vector<DevAbsorb> absorb;
    std::vector<DevPacket> pk;
    std::vector<DevGen> gens;
    std::vector<int *> init_meta;
    std::vector<int *> status_meta;
    for (Req *r : admitted)
        if (r->kind == 1)
            init_meta.push_back(r->slot.meta);
    for (Req *r : sv->active) {
        if (r->kind == 0) {
            if (r->launched)
                continue;
            r->launched = true;
            r->last_step = step;
            gens.push_back(DevGen{r->C, r->S, r->out, r->len, r->ld_s, r->ld, (uint32_t)r->K, (uint32_t)r->N,
                                  nullptr, 0, 1});
            f.enc.push_back(r);
            continue;
        }
        if (r->cancel)
            continue;
        uint32_t n = 0;
        const uint32_t first = (uint32_t)pk.size();
        while (!r->pkts.empty() && (int)n < sv->cfg.burst && r->pkts.front().release <= now) {
            pk.push_back(DevPacket{r->pkts.front().coef, r->pkts.front().payload});
            r->pkts.pop_front();
            n++;
        }
        if (n == 0)
            continue;
        if (sv->cfg.dry_run) {   // scheduling model: every packet is innovative
            const int take = std::min<int>((int)n, r->N - r->rank);
            r->rank += take;
            r->seen += (int)n;
        }
        absorb.push_back(DevAbsorb{r->slot, first, n, (int)step, 0});
        gens.push_back(DevGen{r->slot.Cinv, r->slot.Bsel, r->out, r->len, r->ld, r->ld, (uint32_t)r->N,
                              (uint32_t)r->N, r->slot.meta + 1, (int)step, 1});
        status_meta.push_back(r->slot.meta);
        r->last_step = step;
        f.dec.push_back(r);
    }
    if (absorb.empty() && gens.empty() && init_meta.empty())
        return (int)sv->inflight.size();

    // The step's products run on the matrix cores (bit-matrix form) when every
    // source row starts 4-byte aligned and no packet is too long for it; the
    // table form otherwise.
    bool mf = sv->rows != nullptr;
    for (DevGen &g : gens) {
        g.align = row_align(g.S, g.N > 1 ? g.ld_s : 0, g.Y, g.K > 1 ? g.ld_y : 0);
        if ((((uintptr_t)g.S) | (g.N > 1 ? g.ld_s : 0)) % 4 != 0 || g.len > (1ull << 34))
            mf = false;
    }
    TileQueues tq;
    if (mf)
        build_tiles_mfma(gens.data(), gens.size(), tq);
    else
        build_tiles(gens.data(), gens.size(), 0, tq);
    const std::vector<DevTile> &tiles = tq.tiles;
    std::vector<unsigned> rb = tq.runs;   // runs, then the queue bounds
    rb.insert(rb.end(), tq.bounds, tq.bounds + MF_QUEUES + 1);
    sv->st.steps++;
    sv->st.encode_tiles += tiles.size();
    sv->st.absorb_items += absorb.size();
    sv->st.packets_absorbed += pk.size();
    sv->next_step++;
    sv->next_buf = (sv->next_buf + 1) % (kInflight + 1);

    if (!sv->cfg.dry_run) {
        StepBuf &b = sv->bufs[f.buf];
        const size_t o_abs = 0;
        const size_t o_pk = align16(o_abs + absorb.size() * sizeof(DevAbsorb));
        const size_t o_gen = align16(o_pk + pk.size() * sizeof(DevPacket));
        const size_t o_tile = align16(o_gen + gens.size() * sizeof(DevGen));
        const size_t o_runs = align16(o_tile + tiles.size() * sizeof(DevTile));
        const size_t o_init = align16(o_runs + rb.size() * sizeof(unsigned));
        const size_t o_stat = align16(o_init + init_meta.size() * sizeof(int *));
        const size_t total = align16(o_stat + status_meta.size() * sizeof(int *));
        // the buffer of this ring slot was last used kInflight + 1 steps ago; that step has retired
        if ((rc = ensure_buf(b, total, status_meta.size())))
            return fail(sv, rc);
        memcpy(b.host + o_abs, absorb.data(), absorb.size() * sizeof(DevAbsorb));
        memcpy(b.host + o_pk, pk.data(), pk.size() * sizeof(DevPacket));
        memcpy(b.host + o_gen, gens.data(), gens.size() * sizeof(DevGen));
        memcpy(b.host + o_tile, tiles.data(), tiles.size() * sizeof(DevTile));
        memcpy(b.host + o_runs, rb.data(), rb.size() * sizeof(unsigned));
        memcpy(b.host + o_init, init_meta.data(), init_meta.size() * sizeof(int *));
        memcpy(b.host + o_stat, status_meta.data(), status_meta.size() * sizeof(int *));
        hipStream_t s = sv->stream;
        hipError_t e = hipMemcpyAsync(b.dev, b.host, total, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_meta_init(reinterpret_cast<int *const *>(b.dev + o_init), (int)init_meta.size(), s);
        if (e == hipSuccess)
            e = launch_absorb(reinterpret_cast<const DevAbsorb *>(b.dev + o_abs), (int)absorb.size(),
                              reinterpret_cast<const DevPacket *>(b.dev + o_pk), sv->ptab, sv->inv, s);
        if (e == hipSuccess && !tiles.empty()) {
            const unsigned *runs = reinterpret_cast<const unsigned *>(b.dev + o_runs);
            const DevGen *dg = reinterpret_cast<const DevGen *>(b.dev + o_gen);
            const DevTile *dt = reinterpret_cast<const DevTile *>(b.dev + o_tile);
            if (mf) {
                const int grid = std::max(1, std::min<int>(sv->grid_max_mf, (int)tiles.size()));
                e = launch_encode_mfma(dg, dt, runs, runs + tq.runs.size(), (int)tiles.size(), sv->ctr, grid,
                                       sv->rows, true, s);
            } else {
                const int grid = std::max(1, std::min<int>(sv->grid_max, ((int)tiles.size() + 3) / 4));
                e = launch_encode_persistent(dg, dt, runs, runs + tq.runs.size(), (int)tiles.size(), sv->ctr, grid,
                                             sv->ptab, s);
            }
        }
        if (e == hipSuccess && !status_meta.empty()) {
            e = launch_status_gather(reinterpret_cast<int *const *>(b.dev + o_stat), (int)status_meta.size(),
                                     b.d_status, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b.h_status, b.d_status, status_meta.size() * sizeof(int4),
                                   hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess)
            e = hipEventRecord(b.ev, s);
        if (e != hipSuccess)
            return fail(sv, GF_EDEVICE);
    }
    sv->inflight.push_back(std::move(f));
    return (int)sv->inflight.size();
}

int gf_serve_poll(gf_server *sv, gf_serve_done *out, int max)
{
    if (!sv || max < 0 || (max > 0 && !out))
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    int n = 0;
    while (n < max && !sv->done_fifo.empty()) {
        Req *r = sv->done_fifo.front();
        sv->done_fifo.pop_front();
        r->polled = true;
        gf_serve_done &d = out[n++];
        d.id = r->id;
        d.kind = r->kind;
        d.status = r->status;
        d.rank = r->kind == 1 ? r->rank : r->K;
        d.packets_seen = r->seen;
        d.packets_dropped = r->dropped;
        d.out = r->out;
        d.ld_out = r->ld;
        d.t_submit = r->t_submit;
        d.t_admit = r->t_admit;
        d.t_done = r->t_done;
    }
    return n;
}

int gf_serve_release(gf_server *sv, uint64_t id)
{
    if (!sv)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end() || it->second->state != DONE || !it->second->polled || it->second->release_asked)
        return GF_EINVAL;
    it->second->release_asked = true;
    sv->to_free.push_back(it->second);
    free_ready(sv, retired_step(sv));
    return GF_OK;
}

int gf_serve_query(gf_server *sv, uint64_t id, gf_serve_status *out)
{
    if (!sv || !out)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end() || it->second->release_asked)
        return GF_EINVAL;
    const Req *r = it->second;
    out->state = r->state;
    out->rank = r->kind == 1 ? r->rank : (r->state == DONE ? r->K : 0);
    out->packets_pending = (int)r->pkts.size();
    out->packets_seen = r->seen;
    out->packets_dropped = r->dropped;
    return GF_OK;
}

int gf_serve_cancel(gf_server *sv, uint64_t id, double now)
{
    if (!sv)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end() || it->second->state == DONE || it->second->cancel)
        return GF_EINVAL;
    Req *r = it->second;
    if (r->state == QUEUED) {
        sv->queue.erase(std::remove(sv->queue.begin(), sv->queue.end(), r), sv->queue.end());
        r->state = ACTIVE;   // finish() moves it to the completed list
        finish(sv, r, now, GF_ECANCELED);
        return GF_OK;
    }
    if (r->kind == 0)
        return GF_EINVAL;    // an admitted encode is already in a step: it completes there
    r->cancel = true;
    r->pkts.clear();
    if (r->last_step <= retired_step(sv))
        finish(sv, r, now, GF_ECANCELED);   // no step in flight refers to it
    return GF_OK;
}

int gf_serve_copy_out(gf_server *sv, uint64_t id, uint8_t *dst, size_t ld_dst, void *stream)
{
    if (!sv || !dst)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end() || it->second->state != DONE || it->second->status != GF_OK ||
        it->second->release_asked)
        return GF_EINVAL;
    Req *r = it->second;
    const size_t rows = (size_t)(r->kind == 0 ? r->K : r->N);
    if (rows > 1 && ld_dst < r->len)
        return GF_EINVAL;
    if (sv->cfg.dry_run)
        return GF_OK;
    // the step that produced the output has retired, so the copy only needs
    // to follow the caller's own work; the event after it keeps the memory
    // from being reused (after gf_serve_release) until the copy has run
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return GF_EDEVICE;
    if (hipMemcpy2DAsync(dst, rows > 1 ? ld_dst : r->len, r->out, r->ld, r->len, rows, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream) != hipSuccess ||
        hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return GF_EDEVICE;
    }
    r->copies.push_back(ev);
    return GF_OK;
}

int gf_serve_drain(gf_server *sv, double now)
{
    if (!sv)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err)
        return sv->err;
    while (!sv->inflight.empty()) {
        if (!sv->cfg.dry_run && hipEventSynchronize(sv->bufs[sv->inflight.front().buf].ev) != hipSuccess)
            return fail(sv, GF_EDEVICE);
        retire(sv, now);
    }
    free_ready(sv, retired_step(sv));
    return GF_OK;
}

int gf_serve_stats(gf_server *sv, gf_serve_counters *out)
{
    if (!sv || !out)
        return GF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    out->queued = sv->queue.size();
    out->active = sv->active.size();
    out->inflight_steps = sv->inflight.size();
    out->arena_bytes = sv->arena.size();
    out->arena_used = sv->arena.used();
    out->arena_peak = sv->arena.peak();
    return GF_OK;
}

}  // extern "C"
