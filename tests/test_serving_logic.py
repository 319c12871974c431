"""Admission logic of the serving loop, on a host-only context in dry-run mode.

Dry runs touch no device and write no results: an admitted request "completes"
a fixed time per ray after admission, which lets these tests force queueing,
budget rejection, cancellation, timeouts and ordering from the host.
"""

import time

import pytest


@pytest.fixture()
def L():
    from paper_2504_21627_amd import lsnif
    lsnif.load()
    return lsnif


@pytest.fixture()
def ctx(L):
    c = L.lsnif_create(-1)
    yield c
    L.lsnif_destroy(c)


FAKE = 1 << 20          # a non-null device address; dry runs never dereference it


def req(L, n, timeout_ns=0, object_id=0):
    return L.make_request(rays=FAKE, out=FAKE, n_rays=n, timeout_ns=timeout_ns, object_id=object_id)


def test_host_only_context_refuses_device_work(L, ctx):
    import workloads as W
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_build(ctx, L.ObjectDesc(W.configs.c1_object()))
    assert e.value.status == L.LSNIF_E_DEVICE
    with pytest.raises(L.LsnifError):
        L.lsnif_serve_start(ctx)            # a real serving loop needs a device


def test_all_requests_complete_in_order(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=2, hbm_budget=1 << 30, dry_run_ns_per_ray=2000, merge_max=1)
    tickets = [L.lsnif_serve_submit(ctx, req(L, 64 + 8 * i)) for i in range(20)]
    for t in tickets:
        assert L.lsnif_serve_wait(ctx, t, 10_000_000_000) == L.LSNIF_OK
        assert L.lsnif_serve_poll(ctx, t) == L.LSNIF_REQ_DONE
    s = L.lsnif_serve_stats_get(ctx)
    assert s["completed"] == 20 and s["admitted"] == 20 and s["rays_completed"] == sum(64 + 8 * i for i in range(20))
    assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    L.lsnif_serve_stop(ctx)


def test_slots_limit_concurrency(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=2, hbm_budget=1 << 30, dry_run_ns_per_ray=200_000, merge_max=1)
    ts = [L.lsnif_serve_submit(ctx, req(L, 100)) for _ in range(6)]      # 20 ms each
    time.sleep(0.005)
    s = L.lsnif_serve_stats_get(ctx)
    assert s["inflight"] <= 2 and s["queued"] >= 3
    for t in ts:
        assert L.lsnif_serve_wait(ctx, t) == L.LSNIF_OK
    L.lsnif_serve_stop(ctx)


def dry_ws(n):
    """Workspace of a dry-run query of n rays: the coherence sort at 32^3 cells (2n words,
    262,145 bins, 257 scan partials) when n >= 8192, then a voxel count byte and a list of
    up to 32 voxels per ray, each array 256-byte aligned, then the persistent kernel's
    256-byte tile-queue granule."""
    a = lambda x: (x + 255) // 256 * 256
    sort = a((2 * n + 262_145 + 257) * 4) if n >= 8192 else 0
    return sort + a(n) + a(n * 32 * 4) + 256


def test_budget_rejects_what_can_never_fit_and_queues_the_rest(L, ctx):
    one = dry_ws(100_000)
    L.lsnif_serve_start(ctx, max_inflight=8, hbm_budget=one + 4096, dry_run_ns_per_ray=200, merge_max=1)
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_serve_submit(ctx, req(L, 4_000_000))
    assert e.value.status == L.LSNIF_E_NOMEM
    ts = [L.lsnif_serve_submit(ctx, req(L, 100_000)) for _ in range(3)]   # only one fits at a time
    time.sleep(0.002)
    s = L.lsnif_serve_stats_get(ctx)
    assert s["inflight"] == 1
    for t in ts:
        assert L.lsnif_serve_wait(ctx, t) == L.LSNIF_OK
    s = L.lsnif_serve_stats_get(ctx)
    assert s["rejected"] == 1 and s["completed"] == 3 and s["ws_bytes_peak"] <= one + 4096
    L.lsnif_serve_stop(ctx)


def test_queue_overflow_is_busy(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, max_queue=3, dry_run_ns_per_ray=1_000_000,
                        merge_max=1)
    L.lsnif_serve_submit(ctx, req(L, 50))                    # 50 ms, admitted
    time.sleep(0.005)
    for _ in range(3):
        L.lsnif_serve_submit(ctx, req(L, 1))
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_serve_submit(ctx, req(L, 1))
    assert e.value.status == L.LSNIF_E_BUSY
    assert L.lsnif_serve_stats_get(ctx)["rejected"] == 1
    L.lsnif_serve_stop(ctx)


def test_cancel_waiting_but_not_admitted(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=1_000_000, merge_max=1)
    a = L.lsnif_serve_submit(ctx, req(L, 30))                # admitted, 30 ms
    b = L.lsnif_serve_submit(ctx, req(L, 30))                # waits
    time.sleep(0.005)
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_serve_cancel(ctx, a)
    assert e.value.status == L.LSNIF_E_BUSY
    L.lsnif_serve_cancel(ctx, b)
    assert L.lsnif_serve_poll(ctx, b) == L.LSNIF_E_CANCELLED
    assert L.lsnif_serve_wait(ctx, b) == L.LSNIF_E_CANCELLED
    assert L.lsnif_serve_wait(ctx, a) == L.LSNIF_OK
    s = L.lsnif_serve_stats_get(ctx)
    assert s["cancelled"] == 1 and s["completed"] == 1
    L.lsnif_serve_stop(ctx)


def test_admission_timeout(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=1_000_000, merge_max=1)
    a = L.lsnif_serve_submit(ctx, req(L, 50))                       # 50 ms
    b = L.lsnif_serve_submit(ctx, req(L, 10, timeout_ns=5_000_000))  # gives up after 5 ms in the queue
    assert L.lsnif_serve_wait(ctx, b) == L.LSNIF_E_TIMEOUT
    assert L.lsnif_serve_wait(ctx, a) == L.LSNIF_OK
    assert L.lsnif_serve_stats_get(ctx)["timed_out"] == 1
    L.lsnif_serve_stop(ctx)


def test_wait_timeout_and_unknown_ticket(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=1_000_000, merge_max=1)
    a = L.lsnif_serve_submit(ctx, req(L, 100))                      # 100 ms
    with pytest.raises(L.LsnifError):
        L.lsnif_serve_wait(ctx, a, 1_000_000)
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_serve_poll(ctx, 12345)
    assert e.value.status == L.LSNIF_E_NOTFOUND
    L.lsnif_serve_stop(ctx)


def test_no_overtaking(L, ctx):
    """A large waiting request is not overtaken by small ones that would fit."""
    one = dry_ws(100_000)
    L.lsnif_serve_start(ctx, max_inflight=8, hbm_budget=one + dry_ws(9000) + 8192,
                        dry_run_ns_per_ray=300, merge_max=1)
    big1 = L.lsnif_serve_submit(ctx, req(L, 100_000))               # 30 ms
    big2 = L.lsnif_serve_submit(ctx, req(L, 100_000))               # must wait for big1
    small = L.lsnif_serve_submit(ctx, req(L, 9000))                 # would fit now, but waits behind big2
    time.sleep(0.003)
    assert L.lsnif_serve_poll(ctx, small) == L.LSNIF_REQ_QUEUED
    for t in (big1, big2, small):
        assert L.lsnif_serve_wait(ctx, t) == L.LSNIF_OK
    L.lsnif_serve_stop(ctx)


def test_stop_cancels_waiting(L, ctx):
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=1_000_000, merge_max=1)
    a = L.lsnif_serve_submit(ctx, req(L, 20))
    b = L.lsnif_serve_submit(ctx, req(L, 20))
    time.sleep(0.002)
    L.lsnif_serve_stop(ctx)
    with pytest.raises(L.LsnifError):
        L.lsnif_serve_poll(ctx, a)          # the loop is gone


def _merged(L, ctx, objects, merge_max=0, merge_rays=0, blocker=20):
    """A blocker request (alone: larger than merge_rays) holds the only slot while the
    others queue; returns the stats once all are done."""
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=1_000_000,
                        merge_max=merge_max, merge_rays=merge_rays or 8)
    first = L.lsnif_serve_submit(ctx, req(L, blocker))                  # 20 ms, alone
    time.sleep(0.003)
    ts = [L.lsnif_serve_submit(ctx, req(L, 1, object_id=o)) for o in objects]
    assert L.lsnif_serve_poll(ctx, ts[0]) == L.LSNIF_REQ_QUEUED
    for t in [first] + ts:
        assert L.lsnif_serve_wait(ctx, t, 10_000_000_000) == L.LSNIF_OK
    s = L.lsnif_serve_stats_get(ctx)
    L.lsnif_serve_stop(ctx)
    assert s["completed"] == len(objects) + 1 and s["admitted"] == len(objects) + 1
    assert s["rays_completed"] == blocker + len(objects)
    return s


def test_merging_groups_waiting_neighbours(L, ctx):
    """Ten small requests for one object waiting together run as one launch."""
    assert _merged(L, ctx, [0] * 10)["launches"] == 2


def test_merging_only_joins_the_same_target(L, ctx):
    """Runs of the same object merge; a different object starts a new launch (no
    reordering across targets)."""
    assert _merged(L, ctx, [0, 0, 1, 1, 1, 0, 2])["launches"] == 1 + 4


def test_merging_respects_merge_max_and_merge_rays(L, ctx):
    assert _merged(L, ctx, [0] * 10, merge_max=4)["launches"] == 1 + 3
    assert _merged(L, ctx, [0] * 10, merge_max=1)["launches"] == 1 + 10
    # requests above merge_rays run alone: the blocker itself, here 9 rays with merge_rays 8
    assert _merged(L, ctx, [0] * 3, blocker=9)["launches"] == 2


def test_merged_launch_takes_the_time_of_all_its_rays(L, ctx):
    """In a dry run a merged launch lasts ns_per_ray x its total rays; its members complete
    together."""
    L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=1 << 30, dry_run_ns_per_ray=2_000_000,
                        merge_rays=10)
    first = L.lsnif_serve_submit(ctx, req(L, 11))                       # 22 ms, alone
    time.sleep(0.003)
    ts = [L.lsnif_serve_submit(ctx, req(L, 5)) for _ in range(3)]      # one launch of 15 rays: 30 ms
    assert L.lsnif_serve_wait(ctx, first) == L.LSNIF_OK
    time.sleep(0.010)
    assert all(L.lsnif_serve_poll(ctx, t) == L.LSNIF_REQ_RUNNING for t in ts)
    for t in ts:
        assert L.lsnif_serve_wait(ctx, t) == L.LSNIF_OK
    s = L.lsnif_serve_stats_get(ctx)
    L.lsnif_serve_stop(ctx)
    assert s["launches"] == 2 and s["completed"] == 4
