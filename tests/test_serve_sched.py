"""The serving scheduler without a GPU (dry-run mode: bookkeeping only, every
decode packet counts as innovative): admission by memory budget, FIFO order,
slots, packet release times, deferred release and latency percentiles."""
import pytest

import paper_1909_02871_amd as gf
from paper_1909_02871_amd.serving import percentile

FAKE = 0x7000_0000


def _enc_bytes(K, L):
    ld = (L + 15) // 16 * 16
    return (K * ld + 255) // 256 * 256


def test_admission_respects_budget_and_fifo():
    budget = 64 * 1024
    s = gf.Server(budget_bytes=budget, dry_run=True)
    sizes = [(16, 1500), (8, 4000), (32, 900), (4, 64), (20, 2000), (16, 1500), (2, 9000), (12, 3000)]
    for i, (K, L) in enumerate(sizes):
        s.submit_encode(i, FAKE, FAKE, K, K, L, L, 0.0)
    admitted_order, t = [], 0.0
    while len(admitted_order) < len(sizes):
        t += 0.01
        s.step(t)
        st = s.stats()
        assert st["arena_used"] <= budget
        for d in s.poll():
            admitted_order.append((d["t_admit"], d["id"]))
            s.release(d["id"])
    # admitted in submission order (admission times never decrease with the id)
    ids_by_time = [i for _, i in sorted(admitted_order)]
    assert ids_by_time == sorted(ids_by_time)
    assert s.stats()["arena_peak"] <= budget


def test_head_of_line_request_is_not_starved():
    budget = 40 * 1024
    s = gf.Server(budget_bytes=budget, dry_run=True)
    s.submit_encode(0, FAKE, FAKE, 16, 16, 1500, 1500, 0.0)    # 24 KiB
    s.step(0.0)
    s.submit_encode(1, FAKE, FAKE, 16, 16, 2000, 2000, 0.0)    # 32 KiB: must wait for 0
    s.submit_encode(2, FAKE, FAKE, 1, 1, 64, 64, 0.0)          # tiny, but behind 1 (FIFO)
    s.step(0.1)
    st = s.stats()
    assert st["queued"] == 2
    done = {d["id"]: d for d in s.poll()}
    assert set(done) == {0}
    s.release(0)
    for t in (0.2, 0.3, 0.4):
        s.step(t)
        for d in s.poll():
            done[d["id"]] = d
            s.release(d["id"])
    assert done[1]["t_admit"] <= done[2]["t_admit"]
    assert set(done) == {0, 1, 2}


def test_slots_limit_concurrency():
    s = gf.Server(budget_bytes=1 << 30, max_slots=3, dry_run=True)
    for i in range(10):
        s.submit_decode(i, 8, 100, 0.0)
    s.step(0.0)
    st = s.stats()
    assert st["active"] == 3 and st["queued"] == 7


def test_decode_needs_released_packets():
    s = gf.Server(budget_bytes=1 << 20, burst=3, dry_run=True)
    s.submit_decode(7, 5, 300, 0.0)
    for j in range(5):
        s.push_packet(7, FAKE + j, FAKE + 1000 + j, 0.5 + 0.1 * j)    # released at 0.5 .. 0.9
    for t in (0.0, 0.1, 0.2):
        s.step(t)
        assert s.poll() == []
    assert s.stats()["packets_absorbed"] == 0
    s.step(0.65)          # packets released at 0.5 and 0.6 only
    assert s.stats()["packets_absorbed"] == 2
    s.step(1.0)           # burst 3 of the remaining 3
    s.step(1.1)
    d = s.poll()
    assert len(d) == 1 and d[0]["rank"] == 5 and d[0]["packets_seen"] == 5


def test_burst_limits_packets_per_step():
    s = gf.Server(budget_bytes=1 << 20, burst=4, dry_run=True)
    s.submit_decode(1, 16, 100, 0.0)
    for j in range(16):
        s.push_packet(1, FAKE + j, FAKE + j, 0.0)
    steps = 0
    while not s.poll():
        s.step(1.0 + steps)
        steps += 1
        assert steps < 10
    assert s.stats()["absorb_items"] == 4


def test_release_returns_memory():
    s = gf.Server(budget_bytes=1 << 20, dry_run=True)
    s.submit_encode(1, FAKE, FAKE, 4, 4, 1000, 1000, 0.0)
    s.step(0.0)
    s.step(0.1)
    d = s.poll()
    assert len(d) == 1
    used = s.stats()["arena_used"]
    assert used == _enc_bytes(4, 1000)
    s.release(1)
    assert s.stats()["arena_used"] == 0
    with pytest.raises(gf.GFError):
        s.release(1)


def test_rejects_bad_requests():
    s = gf.Server(budget_bytes=4096, dry_run=True)
    with pytest.raises(gf.GFError) as e:
        s.submit_encode(1, FAKE, FAKE, 64, 64, 9000, 9000, 0.0)     # can never fit
    assert e.value.code == gf.GF_ERANGE
    with pytest.raises(gf.GFError):
        s.submit_decode(2, 0, 100, 0.0)
    with pytest.raises(gf.GFError):
        s.submit_decode(3, 300, 100, 0.0)
    s.submit_decode(4, 4, 10, 0.0)
    with pytest.raises(gf.GFError):
        s.submit_decode(4, 4, 10, 0.0)                            # duplicate id
    with pytest.raises(gf.GFError):
        s.push_packet(99, FAKE, FAKE, 0.0)                        # unknown request


def test_percentiles():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert percentile([5, 1, 4, 2, 3], 50) == 3


def test_release_needs_a_polled_request_and_finished_decodes_take_no_packets():
    s = gf.Server(budget_bytes=1 << 20, dry_run=True)
    s.submit_decode(5, 2, 100, 0.0)
    with pytest.raises(gf.GFError):
        s.release(5)                                  # not completed yet
    for j in range(2):
        s.push_packet(5, FAKE + j, FAKE + j, 0.0)
    s.step(0.0)
    s.step(0.1)
    with pytest.raises(gf.GFError):
        s.release(5)                                  # completed but not polled
    (d,) = s.poll()
    assert d["id"] == 5 and d["rank"] == 2
    with pytest.raises(gf.GFError):
        s.push_packet(5, FAKE, FAKE, 0.2)             # the generation is decoded
    s.release(5)
    assert s.stats()["arena_used"] == 0


def test_calls_from_several_threads_are_serialised():
    import threading

    s = gf.Server(budget_bytes=1 << 30, dry_run=True)
    per_thread, threads = 200, 8

    def work(t):
        for i in range(per_thread):
            rid = t * per_thread + i
            s.submit_decode(rid, 4, 64, 0.0)
            for j in range(4):
                s.push_packet(rid, FAKE + j, FAKE + j, 0.0)

    ws = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for w in ws:
        w.start()
    for w in ws:
        w.join()
    st = s.stats()
    assert st["submitted"] == per_thread * threads
    assert st["packets_pushed"] == 4 * per_thread * threads
    done, t = 0, 0.0
    while done < per_thread * threads:
        t += 1.0
        s.step(t)
        for d in s.poll():
            assert d["rank"] == 4
            s.release(d["id"])
            done += 1
        assert t < 1000
    assert s.stats()["arena_used"] == 0


def test_starved_decode_is_cancelled_and_its_slot_reused():
    """A decode whose sender stops short of rank N never completes by itself;
    cancelling it completes it with GF_ECANCELED (no output), and releasing it
    frees its slot and memory for the request queued behind it."""
    s = gf.Server(budget_bytes=1 << 20, max_slots=1, dry_run=True)
    s.submit_decode(1, 6, 500, 0.0)
    for j in range(4):                       # only 4 of the 6 packets it needs
        s.push_packet(1, FAKE + j, FAKE + 100 + j, 0.0)
    s.submit_decode(2, 3, 500, 0.0)          # waits for the only slot
    for t in (0.1, 0.2, 0.3):
        s.step(t)
        assert s.poll() == []
    st = s.stats()
    assert st["active"] == 1 and st["queued"] == 1
    s.cancel(1, 0.35)
    with pytest.raises(gf.GFError):
        s.push_packet(1, FAKE, FAKE, 0.4)    # a completed request takes no packets
    (d,) = s.poll()
    assert d["id"] == 1 and d["status"] == gf.GF_ECANCELED and d["rank"] == 4
    with pytest.raises(gf.GFError):
        s.cancel(1, 0.4)                     # already completed
    # a cancelled request has no output to copy
    assert gf.lib().gf_serve_copy_out(s._h, 1, 0x1000, 500, None) == gf.GF_EINVAL
    s.release(1)
    for j in range(3):
        s.push_packet(2, FAKE + j, FAKE + 100 + j, 0.4)
    s.step(0.5)
    s.step(0.6)
    (d2,) = s.poll()
    assert d2["id"] == 2 and d2["status"] == gf.GF_OK and d2["rank"] == 3
    assert d2["t_admit"] >= 0.35


def test_cancel_of_queued_requests_and_admitted_encodes():
    s = gf.Server(budget_bytes=64 * 1024, dry_run=True)
    s.submit_encode(1, FAKE, FAKE, 16, 16, 1500, 1500, 0.0)      # 24 KiB
    s.submit_encode(2, FAKE, FAKE, 16, 16, 2000, 2000, 0.0)      # 32 KiB
    s.submit_encode(3, FAKE, FAKE, 16, 16, 2000, 2000, 0.0)      # queued behind the budget
    s.step(0.0)
    assert s.stats()["queued"] == 1
    with pytest.raises(gf.GFError):
        s.cancel(1, 0.01)                     # admitted encode: completes in its step
    s.cancel(3, 0.01)                         # queued: completes at once
    done = {d["id"]: d for d in s.poll()}
    assert done[3]["status"] == gf.GF_ECANCELED and s.stats()["queued"] == 0
    s.step(0.1)
    done.update({d["id"]: d for d in s.poll()})
    assert done[1]["status"] == gf.GF_OK and done[2]["status"] == gf.GF_OK
    with pytest.raises(gf.GFError):
        s.cancel(99, 0.2)                     # unknown id


def test_query_reports_state_and_pending_packets():
    s = gf.Server(budget_bytes=1 << 20, burst=2, max_slots=1, dry_run=True)
    s.submit_decode(1, 4, 100, 0.0)
    s.submit_decode(2, 4, 100, 0.0)
    for j in range(5):
        s.push_packet(1, FAKE + j, FAKE + 100 + j, 0.0)
    assert s.query(1)["state"] == 0 and s.query(1)["packets_pending"] == 5
    s.step(0.1)                      # admitted; takes 2 packets
    q = s.query(1)
    assert q["state"] == 1 and q["packets_pending"] == 3
    s.step(0.2)
    s.step(0.3)
    assert s.query(1)["state"] == 2 and s.query(1)["rank"] == 4
    assert s.query(2)["state"] == 1      # admitted into the slot request 1 left
    (d,) = s.poll()
    s.release(1)
    with pytest.raises(gf.GFError):
        s.query(1)                   # released


def test_replay_cancels_a_starved_decode_only_once_admitted_and_dry():
    """The rateless replay: a decode whose sender runs out before rank N is
    cancelled, but only after the server admitted it and took every packet;
    requests queued behind it for a long time are not."""
    from paper_1909_02871_amd.serving import TraceRequest, replay
    s = gf.Server(budget_bytes=1 << 20, burst=4, max_slots=1, dry_run=True)
    trace = [TraceRequest(0, 0.0, "decode", 6, 100, packets=[(FAKE + j, FAKE + 50 + j, 1e-6 * j) for j in range(3)])]
    trace += [TraceRequest(i, 0.0, "decode", 3, 100, packets=[(FAKE + j, FAKE + 50 + j, 1e-6 * j) for j in range(5)])
              for i in range(1, 4)]
    done = replay(s, trace, timeout_s=20, starve_s=0.2)
    by = {d["id"]: d for d in done}
    assert by[0]["status"] == gf.GF_ECANCELED and by[0]["rank"] == 3
    assert all(by[i]["status"] == gf.GF_OK and by[i]["rank"] == 3 for i in (1, 2, 3))
